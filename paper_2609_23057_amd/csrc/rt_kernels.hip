// Device kernels of the polarized lattice-Boltzmann radiative-transfer solver, gfx950.
//
// State layout: planes p = 4 d + s (direction d, Stokes s), each a row-major
// ny x nx float32 array; plane p starts at p * C, C = nx * ny.  The four
// Stokes planes of a direction are adjacent.
//
// The hot kernel is `fused_kernel`: one time step for a tile of 32
// consecutive cells and all 4n rows (direction x Stokes) of those cells.
// Contraction rows are in the state's own order r = 4 d + s.
//  1. Every wave owns one 32-row tile of the contraction (8 directions x 4
//     Stokes).  The accumulator layout of a 32x32 MFMA tile gives each lane
//     one cell and 16 rows: 4 directions (one per group of 4 accumulator
//     elements) x their 4 Stokes components.  The lane keeps the streaming
//     taps and weights of its 4 directions in registers for the whole
//     kernel, and gathers for them the streamed state (bilinear pull of
//     Eq. 34 from the previous post-collision field, with periodic /
//     absorbing / inflow edges) plus the emission (Eq. 6/8): one tap address
//     per direction serves its 4 Stokes planes.
//  2. The waves write their rows into one LDS tile B[cell][row] in the
//     contraction precision; after a barrier every wave multiplies its 32
//     rows of the collision matrix (pre-swizzled lane fragments read from
//     L2-resident global memory) by the whole B tile on the matrix cores
//     (Eq. 25/30).
//  3. Epilogue in float32: Y = alpha X + beta (M X) (absorption and survival,
//     Sec. 2.1.4-2.1.5, Eq. 11), stored as the next post-collision field.
//
// The adjoint kernel is the same skeleton run backwards: the B tile holds the
// reverse-pulled adjoint field mu = L^T lambda, the matrix-core product uses
// M^T, and the epilogue forms lambda = alpha mu + beta M^T mu together with
// the per-cell gradient contributions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "rt_kernels.h"

namespace rtl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// 16 floats at 16-byte alignment (rows of a matrix whose stride is a multiple of 4 floats)
typedef float f32x16u __attribute__((ext_vector_type(16), aligned(16)));

namespace {

constexpr int kEdgeXp = 1, kEdgeYm = 2, kEdgeYp = 3;

static_assert(sizeof(DirTaps) == 40, "direction tap entry layout");

// Periodic wrap of a source index that lies at most two cells outside [0, n);
// identity on a non-periodic axis.  Branch-free.
__device__ __forceinline__ int wrap_axis(int v, int n, int per) {
  const int m = per ? n : 0;
  v += v < 0 ? m : 0;
  v += v < 0 ? m : 0;
  v -= (per && v >= n) ? m : 0;
  v -= (per && v >= n) ? m : 0;
  return v;
}

// Streaming data of one direction, held by a lane for the whole kernel.
struct LaneDir {
  int64_t off;   // element offset of plane (d, s = 0); Stokes s adds s * C
  int td;        // oy0 * nx + ox0
  int ox0, oy0;  // floor of the displacement (Eq. 34)
  float w00, w10, w01, w11;   // bilinear weights of taps (bx, by)
  int d;         // direction index (rows of padding directions d >= n give zero)
  int oz0;       // 3-D lattice: floor of the z displacement (td then includes it)
};

__device__ __forceinline__ LaneDir lane_dir(const StepArgs &a, int d) {
  LaneDir L;
  L.d = d;
  if (d < a.geo.n) {
    const DirTaps tp = a.taps[d];
    L.off = (int64_t)(4 * d) * a.geo.C;
    L.ox0 = tp.ox0;
    L.oy0 = tp.oy0;
    L.td = tp.oy0 * a.geo.nx + tp.ox0;
    L.w00 = tp.w00;
    L.w10 = tp.w10;
    L.w01 = tp.w01;
    L.w11 = tp.w11;
  } else {
    L.off = 0;
    L.ox0 = L.oy0 = L.td = 0;
    L.w00 = L.w10 = L.w01 = L.w11 = 0.0f;
  }
  return L;
}

// Cell of a lane.  Cell indices fit in 32 bits (nx * ny < 2^31 is validated
// on the host).  Lanes past the end of the lattice take the tile's first cell
// (valid, and interior when the tile is) and are masked to zero.
struct LaneCell {
  int c, x, y;
  bool valid;
  int z;   // layer (3-D lattice; y is then the row within the layer)
};

__device__ __forceinline__ LaneCell lane_cell(const Geometry &g, int c0, int x0, int y0, int col) {
  LaneCell lc;
  lc.valid = (int64_t)c0 + col < g.C;
  int x = x0 + (lc.valid ? col : 0), y = y0;
  while (x >= g.nx) {  // at most ceil(32 / nx) iterations
    x -= g.nx;
    ++y;
  }
  lc.x = x;
  lc.y = y;
  lc.c = y * g.nx + x;
  return lc;
}

// Four-tap pull of Eq. 34.  The forward (REV = false) reads the previous
// post-collision field at (x - ox - bx, y - oy - by); the adjoint (REV = true)
// reads lambda at (x + ox + bx, y + oy + by).  Tap order (bx, by) = (0,0),
// (1,0), (0,1), (1,1).  INTERIOR tiles (every tap of every cell inside the
// lattice, decided once per tile) address the taps from one base.  Elsewhere
// periodic axes wrap, and a tap outside the lattice on a non-periodic axis
// is given its own address in the ghost table instead of the field: the
// ghost radiance of the edge it crossed (forward; a y edge takes precedence
// over an x edge) or the table's zero row (adjoint).  The table is [5][Rpad]
// in row order 4 d + s, so the 4 Stokes values of a direction are adjacent
// there (stride 1) while in the field they are C apart.
struct TapIdx {
  int xs0, xs1, ys0, ys1;
};

template <bool REV>
__device__ __forceinline__ TapIdx tap_index(const Geometry &g, const LaneDir &ld, int x, int y) {
  TapIdx t;
  t.xs0 = wrap_axis(REV ? x + ld.ox0 : x - ld.ox0, g.nx, g.per_x);
  t.xs1 = wrap_axis(REV ? x + ld.ox0 + 1 : x - ld.ox0 - 1, g.nx, g.per_x);
  t.ys0 = wrap_axis(REV ? y + ld.oy0 : y - ld.oy0, g.ny, g.per_y);
  t.ys1 = wrap_axis(REV ? y + ld.oy0 + 1 : y - ld.oy0 - 1, g.ny, g.per_y);
  return t;
}

// Row of the 2-D ghost table a tap outside the lattice reads: the cell of the
// edge it crossed (a y edge takes precedence over an x edge), at its x on a y
// edge (clamped to the lattice at the corners) or its y on an x edge; rows
// run x- (y = 0..ny-1), x+, y- (x = 0..nx-1), y+, then one row of zeros.
__device__ __forceinline__ int ghost_row(const Geometry &g, int xs, int ys, bool iny) {
  const int gx = min(max(xs, 0), g.nx - 1);
  return !iny ? 2 * g.ny + (ys < 0 ? 0 : g.nx) + gx : (xs < 0 ? 0 : g.ny) + ys;
}
__device__ __forceinline__ int ghost_zero_row(const Geometry &g) { return 2 * (g.nx + g.ny); }

template <bool REV>
__device__ __forceinline__ void edge_taps(const StepArgs &a, const float *__restrict__ src,
                                          const Geometry &g, const LaneDir &ld, const LaneCell &lc,
                                          const float *(&p)[4], int (&stride)[4]) {
  const TapIdx t = tap_index<REV>(g, ld, lc.x, lc.y);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int xs = (k & 1) ? t.xs1 : t.xs0;
    const int ys = (k & 2) ? t.ys1 : t.ys0;
    const bool inx = (unsigned)xs < (unsigned)g.nx, iny = (unsigned)ys < (unsigned)g.ny;
    const bool inside = inx && iny;
    const int row = REV ? ghost_zero_row(g) : ghost_row(g, xs, ys, iny);
    // branch-free: one base pointer select and one offset select
    const float *base = inside ? src : a.ghost;
    const int64_t eoff = inside ? ld.off + (ys * g.nx + xs) : (int64_t)row * g.Rpad + 4 * ld.d;
    p[k] = base + eoff;
    stride[k] = inside ? (int)g.C : 1;
  }
}

// Bilinear combination of the 4 taps of one plane.  Device code is built
// without automatic multiply-add contraction; the fused multiply-adds are
// written out so that every kernel instantiation rounds identically.
__device__ __forceinline__ float tap_sum(const LaneDir &ld, const float (&v)[4]) {
  return fmaf(ld.w10, v[1], ld.w00 * v[0]) + fmaf(ld.w11, v[3], ld.w01 * v[2]);
}

// One group = the 4 Stokes rows of one of the lane's directions: their 16
// tap loads (or 4 direct loads) are issued together.
template <bool REV, bool GATHER, bool INTERIOR>
__device__ __forceinline__ void dir_issue(const StepArgs &a, const float *__restrict__ src,
                                          const Geometry &g, const LaneDir &ld, const LaneCell &lc,
                                          float (&v)[4][4]) {
  if (!GATHER) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      v[s][0] = src[ld.off + (int64_t)s * g.C + lc.c];
      v[s][1] = v[s][2] = v[s][3] = 0.0f;
    }
  } else if (INTERIOR) {
    const int step = REV ? 1 : -1;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float *p0 = src + ld.off + (int64_t)s * g.C + lc.c + (REV ? ld.td : -ld.td);
      const float *p1 = p0 + step * g.nx;
      v[s][0] = p0[0];
      v[s][1] = p0[step];
      v[s][2] = p1[0];
      v[s][3] = p1[step];
    }
  } else {
    const float *p[4];
    int stride[4];
    edge_taps<REV>(a, src, g, ld, lc, p, stride);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[s][k] = p[k][(int64_t)s * stride[k]];
  }
}

// Combines a group into dst[0..3] (the 4 Stokes of the direction): the pulled
// (or direct) value, plus dt_pre * eps * j[d][s] for the state field (EMIT;
// jrow is the block's LDS copy of the emission rows, so that reading it never
// waits on the wave's outstanding global loads); for CKPT the streamed value
// before emission is also stored into s_out.
// Dichroic factor of one direction on (I, Q): I + Q scaled by exp(-x) and
// I - Q by exp(x), written as I cosh x - Q sinh x and Q cosh x - I sinh x so
// that a small Q is not the difference of two intensity-sized terms.
__device__ __forceinline__ void dich_factor(float &xI, float &xQ, float x) {
  const float ch = coshf(x), sh = sinhf(x);
  const float i = xI, q = xQ;
  xI = fmaf(-q, sh, i * ch);
  xQ = fmaf(-i, sh, q * ch);
}

template <bool GATHER, bool EMIT, bool CKPT, bool DICH = false>
__device__ __forceinline__ void dir_combine(const StepArgs &a, const Geometry &g, const LaneDir &ld,
                                            const LaneCell &lc, float emis_dt, const float (&v)[4][4],
                                            float *dst, const float *jrow, float xi = 0.0f, float wd = 0.0f) {
  const bool live = lc.valid && ld.d < g.n;
  f32x4 jp = f32x4{0.f, 0.f, 0.f, 0.f};
  if (EMIT) jp = *reinterpret_cast<const f32x4 *>(jrow + 4 * ld.d);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    float sv = v[s][0];
    if (GATHER) sv = tap_sum(ld, v[s]);
    if (CKPT && live) a.s_out[ld.off + (int64_t)s * g.C + lc.c] = sv;
    if (EMIT) sv = fmaf(emis_dt, jp[s], sv);
    dst[s] = live ? sv : 0.0f;
  }
  if constexpr (DICH) {
    // dichroic absorption: the linear polarisations along e_theta (I + Q)
    // and e_phi (I - Q) decay at their own rates exp(-+xi w_d); the common
    // factor exp(-tau_abs) is in alpha and beta
    dich_factor(dst[0], dst[1], xi * wd);
  }
}

// Gathers the 16 values a lane owns: the streamed (GATHER) or direct state
// with emission, or with REV the reverse-pulled adjoint field.  Group k (the
// 4 Stokes rows of direction 8 t + 2 k + h) goes to dst[4k..4k+3], or with
// an LDS destination (put_group) as soon as it is combined, so that it holds
// no registers afterwards.  Interior tiles run a
// two-stage pipeline (group k's loads are issued before group k-1 is
// combined: two groups, 32 loads, in flight); edge tiles take one group at a
// time.
// Where a combined group goes: registers dst[4k..4k+3], the float32 X tile
// (lds = the lane's first row there, rows 8 k apart = 32 k bytes), or split
// into a bf16 high part (lds = the lane's first row of the B tile, 16 k
// bytes) and the low part v - high (lo_off bytes further: the low tile).
enum { kPutReg = 0, kPutF32 = 1, kPutSplit = 2 };

template <int PUT>
__device__ __forceinline__ void put_group(const float (&o)[4], float *dst, char *lds, int k, int lo_off) {
  if (PUT == kPutF32) {
    *reinterpret_cast<f32x4 *>(lds + 32 * k) = f32x4{o[0], o[1], o[2], o[3]};
  } else if (PUT == kPutSplit) {
    bf16x4 hv, lv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hv[j] = static_cast<__bf16>(o[j]);
      lv[j] = static_cast<__bf16>(o[j] - static_cast<float>(hv[j]));
    }
    *reinterpret_cast<bf16x4 *>(lds + 16 * k) = hv;
    *reinterpret_cast<bf16x4 *>(lds + lo_off + 16 * k) = lv;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) dst[4 * k + s] = o[s];
  }
}

// The emission factor dt_pre * eps of the cell is formed only once the first
// group's loads are issued: eps comes from a load issued just before, and
// loads and stores complete in issue order, so using it earlier would make
// the tile wait for the previous tile's stores before its first gather load.
__device__ __forceinline__ float late_emission(const StepArgs &a, float emis) {
  asm volatile("" : "+v"(emis));
  return a.dt_pre * emis;
}

template <bool REV, bool GATHER, bool INTERIOR, bool EMIT, bool CKPT, int PUT, bool DICH = false>
__device__ __forceinline__ void gather_field(const StepArgs &a, const float *__restrict__ src,
                                             const Geometry &g, const LaneDir (&ld)[4],
                                             const LaneCell &lc, float emis, float *dst,
                                             char *lds, const float *jrow, int lo_off = 0, float xi = 0.0f,
                                             const float *wd = nullptr) {
  float emis_dt = 0.0f;
  if (!INTERIOR) {
    // edge tiles (a small share): one group at a time, which keeps the wrap
    // and ghost bookkeeping of only one direction live
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float v[4][4], o[4];
      dir_issue<REV, GATHER, INTERIOR>(a, src, g, ld[k], lc, v);
      if (EMIT && k == 0) emis_dt = late_emission(a, emis);
      dir_combine<GATHER, EMIT, CKPT, DICH>(a, g, ld[k], lc, emis_dt, v, o, jrow, xi, DICH ? wd[k] : 0.0f);
      put_group<PUT>(o, dst, lds, k, lo_off);
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  float va[4][4], vb[4][4];
  dir_issue<REV, GATHER, INTERIOR>(a, src, g, ld[0], lc, va);
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    if (k < 4) dir_issue<REV, GATHER, INTERIOR>(a, src, g, ld[k], lc, vb);
    __builtin_amdgcn_sched_barrier(0);
    if (EMIT && k == 1) emis_dt = late_emission(a, emis);
    float o[4];
    dir_combine<GATHER, EMIT, CKPT, DICH>(a, g, ld[k - 1], lc, emis_dt, va, o, jrow, xi,
                                          DICH ? wd[k - 1] : 0.0f);
    put_group<PUT>(o, dst, lds, k - 1, lo_off);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < 4; ++m) va[j][m] = vb[j][m];
  }
}

// ---- 3-D lattice: the trilinear pull (Eq. 34 along x, y and z) in the gather
// Tap b = bx + 2 by + 4 bz of direction d reads the previous post-collision
// field at (x - ox0 - bx, y - oy0 - by, z - oz0 - bz) with weight w_b (the
// direction's 8 weights, from the block's LDS copy).  The taps are summed in
// increasing b with one fused multiply-add each, as the stand-alone 3-D
// streaming kernel sums them, so that a fused step reproduces collision then
// streaming bit for bit.  A tap outside the lattice on a non-periodic axis
// reads the face table (z faces before y faces before x faces).

__device__ __forceinline__ LaneDir lane_dir3(const StepArgs &a, int d) {
  LaneDir L{};
  L.d = d;
  if (d < a.geo.n) {
    const DirTaps3 tp = a.taps3[d];
    L.off = (int64_t)(4 * d) * a.geo.C;
    L.ox0 = tp.ox0;
    L.oy0 = tp.oy0;
    L.oz0 = tp.oz0;
    L.td = (tp.oz0 * a.ny3 + tp.oy0) * a.geo.nx + tp.ox0;
  }
  return L;
}

// Row (y, z) and first column x0 of 3-D tile `tile` (tiles of `cells` cells
// never span rows): rows are taken in blocks of zblk layers, the layer index
// fastest within a block, so that the rows a tile's taps share with its
// neighbours in z are read again while still in the XCD's L2.
__device__ __forceinline__ void tile_row3(const StepArgs &a, int tile, int cells, int &x0, int &y, int &z) {
  const int tpr = (a.geo.nx + cells - 1) / cells;
  const int w = tile / tpr;
  const int xt = tile - w * tpr;
  const int blk = a.ny3 * a.zblk;
  const int zb = w / blk;
  const int r = w - zb * blk;
  const int zl = min(a.zblk, a.nz - zb * a.zblk);
  y = r / zl;
  z = zb * a.zblk + (r - y * zl);
  x0 = xt * cells;
}

__device__ __forceinline__ float tap_sum3(const f32x4 &w0, const f32x4 &w1, const float (&v)[8]) {
  float acc = 0.0f;
#pragma unroll
  for (int b = 0; b < 4; ++b) acc = fmaf(w0[b], v[b], acc);
#pragma unroll
  for (int b = 0; b < 4; ++b) acc = fmaf(w1[b], v[4 + b], acc);
  return acc;
}

// The 8 tap addresses of one direction at an edge cell: the field (stride C
// between Stokes planes) or the face table (stride 1).
__device__ __forceinline__ void edge_taps3(const StepArgs &a, const float *__restrict__ src, const LaneDir &ld,
                                           const LaneCell &lc, const float *(&p)[8], int (&stride)[8]) {
  const Geometry &g = a.geo;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int xs = wrap_axis(lc.x - ld.ox0 - (b & 1), g.nx, g.per_x);
    const int ys = wrap_axis(lc.y - ld.oy0 - ((b >> 1) & 1), a.ny3, g.per_y);
    const int zs = wrap_axis(lc.z - ld.oz0 - (b >> 2), a.nz, a.per_z);
    const bool inx = (unsigned)xs < (unsigned)g.nx, iny = (unsigned)ys < (unsigned)a.ny3,
               inz = (unsigned)zs < (unsigned)a.nz;
    const bool inside = inx && iny && inz;
    const int f = !inz ? (zs < 0 ? 4 : 5) : (!iny ? (ys < 0 ? 2 : 3) : (xs < 0 ? 0 : 1));
    const float *base = inside ? src : a.ghost;
    const int64_t eoff = inside ? ld.off + ((zs * a.ny3 + ys) * g.nx + xs) : (int64_t)f * g.Rpad + 4 * ld.d;
    p[b] = base + eoff;
    stride[b] = inside ? (int)g.C : 1;
  }
}

// Interior taps of Stokes components s0 and s0 + 1 of one direction (every
// tap of the tile inside the lattice): 16 loads from one base.
__device__ __forceinline__ void dir3_issue_half(const StepArgs &a, const float *__restrict__ src, const LaneDir &ld,
                                                const LaneCell &lc, int s0, float (&v)[2][8]) {
  const int nx = a.geo.nx, lay = a.geo.nx * a.ny3;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float *p = src + ld.off + (int64_t)(s0 + j) * a.geo.C + (lc.c - ld.td);
#pragma unroll
    for (int b = 0; b < 8; ++b) v[j][b] = p[-((b & 1) + ((b >> 1) & 1) * nx + (b >> 2) * lay)];
  }
}

// Taps of Stokes s0 and s0 + 1 of one direction in a tile whose rows are all
// inside in y and z ("row" tiles): x wraps on a periodic axis; a tap outside
// in x is loaded from the lane's own cell (a valid address) and replaced by
// its face's ghost value when summed (row_fix).
__device__ __forceinline__ void dir3_issue_row(const StepArgs &a, const float *__restrict__ src, const LaneDir &ld,
                                               const LaneCell &lc, int s0, float (&v)[2][8]) {
  const Geometry &g = a.geo;
  const int xs0 = wrap_axis(lc.x - ld.ox0, g.nx, g.per_x), xs1 = wrap_axis(lc.x - ld.ox0 - 1, g.nx, g.per_x);
  const int xa0 = (unsigned)xs0 < (unsigned)g.nx ? xs0 : lc.x;
  const int xa1 = (unsigned)xs1 < (unsigned)g.nx ? xs1 : lc.x;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float *p = src + ld.off + (int64_t)(s0 + j) * g.C;
#pragma unroll
    for (int r = 0; r < 4; ++r) {   // r = by + 2 bz
      const int row = ((lc.z - ld.oz0 - (r >> 1)) * a.ny3 + (lc.y - ld.oy0 - (r & 1))) * g.nx;
      v[j][2 * r] = p[row + xa0];
      v[j][2 * r + 1] = p[row + xa1];
    }
  }
}

// Replaces the taps of a row tile that lie outside in x by the ghost value
// of their face (gx: the block's LDS copy of the x- and x+ face rows).
__device__ __forceinline__ void row_fix(const StepArgs &a, const LaneDir &ld, const LaneCell &lc, int s,
                                        const float *gx, float (&v)[8]) {
  const int nx = a.geo.nx;
  const int xs0 = wrap_axis(lc.x - ld.ox0, nx, a.geo.per_x), xs1 = wrap_axis(lc.x - ld.ox0 - 1, nx, a.geo.per_x);
  const float g0 = gx[(xs0 < 0 ? 0 : a.geo.Rpad) + 4 * ld.d + s];
  const float g1 = gx[(xs1 < 0 ? 0 : a.geo.Rpad) + 4 * ld.d + s];
  const bool in0 = (unsigned)xs0 < (unsigned)nx, in1 = (unsigned)xs1 < (unsigned)nx;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    v[2 * r] = in0 ? v[2 * r] : g0;
    v[2 * r + 1] = in1 ? v[2 * r + 1] : g1;
  }
}

// Tile kinds of the 3-D gather: every tap of every cell inside; rows inside
// in y and z (taps may leave in x); anything else.
enum { kG3Edge = 0, kG3Row = 1, kG3Interior = 2 };

// The 3-D counterpart of gather_field (forward state only): the 16 values of
// a lane, pulled trilinearly, with emission, into registers or LDS as
// put_group places them.  Interior and row tiles run a two-stage pipeline
// over half groups (two Stokes planes, 16 loads: the next half's loads are
// issued before the previous half is summed); edge tiles take one direction
// at a time.  w3: the block's LDS copy of the tap weights [Rpad / 4][8],
// followed by the x- and x+ face rows of the ghost table.
template <int MODE, bool CKPT, int PUT, bool DICH = false>
__device__ __forceinline__ void gather_field3(const StepArgs &a, const float *__restrict__ src,
                                              const LaneDir (&ld)[4], const LaneCell &lc, float emis, float *dst,
                                              char *lds, const float *jrow, const float *w3, int lo_off = 0,
                                              float xi = 0.0f, const float *wd = nullptr) {
  const Geometry &g = a.geo;
  float emis_dt = 0.0f;
  auto weights = [&](int k, f32x4 &w0, f32x4 &w1) {
    w0 = *reinterpret_cast<const f32x4 *>(w3 + 8 * ld[k].d);
    w1 = *reinterpret_cast<const f32x4 *>(w3 + 8 * ld[k].d + 4);
  };
  if (MODE == kG3Edge) {
    // (a small share of the tiles: one Stokes plane of one direction at a
    // time, which keeps the register peak of this path below the others')
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float *p[8];
      int stride[8];
      edge_taps3(a, src, ld[k], lc, p, stride);
      if (k == 0) emis_dt = late_emission(a, emis);
      f32x4 w0, w1;
      weights(k, w0, w1);
      float t[4][4] = {};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) v[b] = p[b][(int64_t)s * stride[b]];
        t[s][0] = tap_sum3(w0, w1, v);
        __builtin_amdgcn_sched_barrier(0);
      }
      float o[4];
      dir_combine<false, true, CKPT, DICH>(a, g, ld[k], lc, emis_dt, t, o, jrow, xi, DICH ? wd[k] : 0.0f);
      put_group<PUT>(o, dst, lds, k, lo_off);
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  float va[2][8], vb[2][8];
  float t[4][4] = {};
  auto issue = [&](int k, int s0, float (&v)[2][8]) {
    if (MODE == kG3Interior)
      dir3_issue_half(a, src, ld[k], lc, s0, v);
    else
      dir3_issue_row(a, src, ld[k], lc, s0, v);
  };
  issue(0, 0, va);
#pragma unroll
  for (int u = 1; u <= 8; ++u) {
    if (u < 8) issue(u >> 1, 2 * (u & 1), vb);
    __builtin_amdgcn_sched_barrier(0);
    if (u == 1) emis_dt = late_emission(a, emis);
    const int k = (u - 1) >> 1, hf = (u - 1) & 1;
    f32x4 w0, w1;
    weights(k, w0, w1);
    if (MODE == kG3Row) {
      const float *gx = w3 + 2 * g.Rpad;
      row_fix(a, ld[k], lc, 2 * hf, gx, va[0]);
      row_fix(a, ld[k], lc, 2 * hf + 1, gx, va[1]);
    }
    t[2 * hf][0] = tap_sum3(w0, w1, va[0]);
    t[2 * hf + 1][0] = tap_sum3(w0, w1, va[1]);
    if (hf == 1) {
      float o[4];
      dir_combine<false, true, CKPT, DICH>(a, g, ld[k], lc, emis_dt, t, o, jrow, xi, DICH ? wd[k] : 0.0f);
      put_group<PUT>(o, dst, lds, k, lo_off);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int b = 0; b < 8; ++b) va[j][b] = vb[j][b];
  }
}

// First cell of 2-D tile `tile` (tiles of `cells` consecutive cells).  In
// row order the tiles run through the lattice cell by cell; in strip order
// (a.strip tiles wide, nx a multiple of cells * a.strip) they walk down a
// vertical strip row by row, so the rows of all 4n planes that the tiles in
// flight share with the next output rows stay within a few MB of L2.
__device__ __forceinline__ int tile_cell0(const StepArgs &a, int64_t tile, int cells) {
  const int w = a.strip;
  if (w <= 0) return (int)(tile * cells);
  const int nx = a.geo.nx, ny = a.geo.ny;
  const int t = (int)tile;
  const int per_strip = w * ny;
  const int sidx = t / per_strip, r = t - sidx * per_strip;
  const int y = r / w, xt = sidx * w + (r - y * w);
  return y * nx + xt * cells;
}

// Row r of the 32x32 accumulator held by element i of a lane in half-wave h.
__device__ __forceinline__ int acc_row(int i, int h) { return (i >> 2) * 8 + h * 4 + (i & 3); }

template <int PREC> struct PrecTraits;
// esize: bytes per B-tile element; ntile: B tiles (bf16x3 keeps high and low parts)
template <> struct PrecTraits<P_F32> { static constexpr int esize = 4, ntile = 1; };
template <> struct PrecTraits<P_BF16> { static constexpr int esize = 2, ntile = 1; };
template <> struct PrecTraits<P_F16> { static constexpr int esize = 2, ntile = 1; };
template <> struct PrecTraits<P_BF16X3> { static constexpr int esize = 2, ntile = 2; };

struct LdsLayout {
  int b_off, x_off, red_off;   // within a tile group
  int group;                   // bytes of one tile group; group g starts at g * group
  int jrow_off, total;         // block-wide
  int w3_off;                  // 3-D gather: tap weights [Rpad / 4][8], x face rows [2][Rpad] (block-wide)
  int strideB;   // bytes per cell row of the B tile
  int tileB;     // bytes of one B tile
  int strideX;   // bytes per cell row of the float32 X tile
};

// LDS of a fused launch, per tile group (the W waves that share one tile of
// 32 nb cells): the B tile(s) [32 nb cells][Rpad rows] (row stride padded by
// 16 bytes against bank conflicts of the 16-byte fragment reads), a float32
// tile of the forward operand X [32 nb cells][Rpad rows] that the gather
// writes and the epilogue reads back (the B tile itself for the forward
// float32 contraction), and the cross-wave reduction scratch (fp16 scales,
// adjoint per-cell sums).  After the groups, one copy of the emission rows.
// With xsplit (nb = 2, a bf16 contraction in 16-wave blocks, where a float32
// X tile would not fit beside the B tile), X is not kept in float32: it is
// held as a high part (the B tile) and a low part (a second tile of the same
// shape) whose sum restores it to 2^-18.
__host__ __device__ inline LdsLayout lds_layout(int Rpad, int esize, int ntile, int W, bool adjoint,
                                               bool f16, int ngroups = 1, int nb = 1, int nacc = 3,
                                               bool w3 = false, bool xsplit = false) {
  LdsLayout L;
  // the bf16 / bf16x3 adjoint keeps mu as high (B) and low tiles
  const bool musplit = adjoint && esize == 2 && !f16;
  int off = 0;
  L.b_off = off;
  L.strideB = Rpad * esize + 16;
  L.tileB = 32 * nb * L.strideB;
  off += ((xsplit || musplit) ? 2 : ntile) * L.tileB;
  // the forward float32 contraction reads X itself: the X tile is the B tile
  L.strideX = Rpad * 4 + 16;
  if (!xsplit && (adjoint || esize != 4)) {
    L.x_off = off;
    off += 32 * nb * L.strideX;
  } else {
    L.x_off = L.b_off;
  }
  L.red_off = off;
  const int nred = adjoint ? nacc : (f16 ? 1 : 0);   // adjoint: nacc per-cell sums
  off += nred * W * 32 * nb * 4;
  L.group = off;
  L.jrow_off = ngroups * off;
  L.total = L.jrow_off + Rpad * 4;
  // 3-D gather: the 8 tap weights of each of the Rpad / 4 directions, then
  // the x- and x+ face rows of the ghost table
  L.w3_off = L.total;
  if (w3) L.total += Rpad * 8 + Rpad * 8;
  return L;
}

// Cells per tile of a single-problem step: 64 (two 32-cell column blocks
// that share every A fragment) for the float32 forward step and for the bf16
// forward step with at most 4 row tiles (n <= 32) or more than 8 (n > 64);
// 32 otherwise (bf16x3 needs its float32 X tile, fp16 the whole cell for its
// scale before it can split X, and bf16 at 32 < n <= 64 keeps the float32 X
// tile, which two column blocks of 8 row tiles would hold at one block per
// CU).  Up to 4 row tiles the 64-cell tile performs the 32-cell tile's
// arithmetic per cell, so the spectral batch's 32-cell tiles give the same
// bits.
template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

// Single-problem forward steps with a non-temporal copy of the epilogue: the
// 64-cell tiles, the 16-wave blocks and the 3-D step, without extensions
// (the 32-cell tiles of 4-wave blocks hold no registers to spare for it).
template <bool ADJ, int MAXW, int NB, int EXT, bool G3>
constexpr bool kNtCopy = !ADJ && EXT == kExtNone && (MAXW > 4 || NB > 1 || G3);

// X as high + low bf16 tiles: the bf16 64-cell tile of the 16-wave blocks.
template <int PREC, int MAXW, int NB>
constexpr bool kXSplit = NB > 1 && PREC == P_BF16 && MAXW > 4;

__host__ __device__ inline int step_nb(int W, int prec, bool adjoint) {
  return (!adjoint && (prec == P_F32 || (prec == P_BF16 && (W <= 4 || W > 8)))) ? 2 : 1;
}

// Lane-record offset (before adding the lane) of the A fragments of K step s
// of a tile: the table's zero block for steps past the tile's range.
__device__ __forceinline__ int frag_rec(const TileRange &tr, int s, int nk) {
  return s < nk ? tr.frag_off + s * 64 : tr.zero_off;
}

__device__ __forceinline__ f32x16 mfma_step_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// One 32-cell tile of the fused step, executed by the W waves of one tile
// group (this wave: row tile t = wg).  An inactive group (no tile left in a
// ragged batch) still takes part in every barrier; its lanes count as
// invalid, read the lattice's first cells and store nothing.
struct TileLds {
  char *s_b, *s_x;
  float *s_red;
  const float *s_jrow;
  const float *s_w3;   // 3-D gather: tap weights
};

// Per-cell power-of-two scale of the fp16 operand: 2^(8 - e) for the largest
// |value| m = f 2^e of the cell over all rows (all waves of the group, via
// LDS scratch red[W][32]); 1 for an all-zero cell.
__device__ __forceinline__ float f16_cell_scale(const float (&v)[16], float *red, int wg, int W, int col, int h) {
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) m = fmaxf(m, fabsf(v[i]));
  m = fmaxf(m, __shfl_xor(m, 32));
  if (h == 0) red[wg * 32 + col] = m;
  __syncthreads();
  m = 0.0f;
  for (int ww = 0; ww < W; ++ww) m = fmaxf(m, red[ww * 32 + col]);
  int e = 0;
  if (m > 0.0f) (void)frexpf(m, &e);
  return (m > 0.0f) ? ldexpf(1.0f, 8 - e) : 1.0f;
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT, int kRing, int NB = 1, int EXT = kExtNone, bool G3 = false,
          bool XSPLIT = false, bool NTC = false>
__device__ __forceinline__ void fused_tile(const StepArgs &a, const Geometry &g, const LdsLayout &L,
                                           const TileLds &ts, const TileRange &tr, const LaneDir (&ld)[4],
                                           int64_t tile, bool active, int t, int wg, int W, int lane) {
  static_assert(NB == 1 || (NB == 2 && !ADJ && (PREC == P_F32 || PREC == P_BF16)),
                "two column blocks: forward float32 or bf16");
  constexpr bool MIX = EXT == kExtMix;
  constexpr bool DICH = EXT == kExtDich;
  static_assert(!MIX || NB == 1, "phase mixtures: one column block");
  static_assert(!DICH || !ADJ || NB == 1, "dichroic absorption in the adjoint: one column block");
  static_assert(!G3 || (GATHER && !ADJ && EXT == kExtNone), "3-D gather: forward step without extensions");
  // adjoint per-cell sums: <mu, X_d>, <nu, X_d>, the emission term, and with
  // dichroic absorption the xi-derivative term
  constexpr int NACC = (ADJ && DICH) ? 4 : 3;
  // XSPLIT (bf16 contraction with two column blocks in 16-wave blocks): X
  // lives as high + low tiles; otherwise X is a float32 tile
  static_assert(!XSPLIT || (NB > 1 && PREC == P_BF16), "X split: bf16 with two column blocks");
  const int col = lane & 31;
  const int h = lane >> 5;
  char *s_b = ts.s_b;
  char *s_x = ts.s_x;
  float *s_red = ts.s_red;
  const float *s_jrow = ts.s_jrow;
  (void)s_red;
  (void)s_x;
  const int c0 = active ? tile_cell0(a, tile, 32 * NB) : 0;
  // adjoint mu in registers: only for fp16, whose per-cell scale needs the
  // whole cell before mu can be converted (fp32 gathers mu into its B tile,
  // bf16 and bf16x3 into high and low 16-bit tiles)
  constexpr bool MUSPLIT = ADJ && (PREC == P_BF16 || PREC == P_BF16X3);
  float mv[ADJ && PREC == P_F16 ? 16 : 1];
  float cscale[NB];
  (void)mv;
  // this lane's rows in the LDS tiles: cell 32 cb + col, rows rbase + 8 q + (0..3)
  const int rbase = t * 32 + h * 4;

  // adjoint: the float64 accumulator this lane updates first at the end of
  // the tile (entry e = wg * 64 + lane of the NACC x 32 per-cell sums),
  // loaded now so that its latency is hidden under the tile
  double gpre = 0.0;
  if constexpr (ADJ) {
    const int e = wg * 64 + lane;
    const int k = e / 32, cc = e - k * 32;
    if (e < NACC * 32 && active && (int64_t)c0 + cc < g.C) gpre = a.gacc[(int64_t)k * g.C + c0 + cc];
  }

  // ---- 1. gather own rows, per 32-cell column block --------------------------
  LaneCell lcs[NB];
  bool inter[NB];
  float al[NB], be[NB], em[NB];
  float fr[MIX ? NB : 1];   // phase mixture: weight of the first matrix, 1 - sum of the fractions
  float f0[MIX ? NB : 1];   // and the first further matrix's fraction
  (void)fr;
  float xi[DICH ? NB : 1];  // dichroic absorption: tau_abs * eta of the cell
  float wdir[DICH ? 4 : 1]; // and sin^2 theta of the lane's four directions
  (void)xi;
  (void)wdir;
  if constexpr (DICH) {
#pragma unroll
    for (int q = 0; q < 4; ++q) wdir[q] = (a.dich_w != nullptr && ld[q].d < g.n) ? a.dich_w[ld[q].d] : 0.0f;
  }
  if constexpr (G3) {
    // 3-D lattice: the tile is the cells x0 .. x0 + 32 NB - 1 of one row
    // (y, z); lanes past the row's end take its first cell and are masked
    int x0, y3, z3;
    tile_row3(a, active ? (int)tile : 0, 32 * NB, x0, y3, z3);
    const int rowc = (z3 * a.ny3 + y3) * g.nx;
    const bool yz_in = y3 >= 2 && y3 <= a.ny3 - 3 && z3 >= 2 && z3 <= a.nz - 3;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      cscale[cb] = 1.0f;
      const int xb = x0 + 32 * cb;
      LaneCell lc;
      lc.valid = active && xb + col < g.nx;
      lc.x = lc.valid ? xb + col : x0;
      lc.y = y3;
      lc.z = z3;
      lc.c = rowc + lc.x;
      lcs[cb] = lc;
      al[cb] = a.alpha[lc.c];
      be[cb] = a.beta[lc.c];
      em[cb] = a.emis[lc.c];
      // every tap of every cell inside the lattice (taps reach two cells),
      // or at least every row of the tile's taps
      const bool interior = yz_in && xb >= 2 && xb + 31 <= g.nx - 3;
      inter[cb] = interior;
      if constexpr (XSPLIT) {
        char *brow = s_b + (32 * cb + col) * L.strideB + rbase * 2;
        if (interior)
          gather_field3<kG3Interior, CKPT, kPutSplit>(a, a.in, ld, lc, em[cb], nullptr, brow, s_jrow, ts.s_w3,
                                                      L.tileB);
        else if (yz_in)
          gather_field3<kG3Row, CKPT, kPutSplit>(a, a.in, ld, lc, em[cb], nullptr, brow, s_jrow, ts.s_w3, L.tileB);
        else
          gather_field3<kG3Edge, CKPT, kPutSplit>(a, a.in, ld, lc, em[cb], nullptr, brow, s_jrow, ts.s_w3, L.tileB);
      } else {
        char *xrow = s_x + (32 * cb + col) * L.strideX + rbase * 4;
        if (interior)
          gather_field3<kG3Interior, CKPT, kPutF32>(a, a.in, ld, lc, em[cb], nullptr, xrow, s_jrow, ts.s_w3);
        else if (yz_in)
          gather_field3<kG3Row, CKPT, kPutF32>(a, a.in, ld, lc, em[cb], nullptr, xrow, s_jrow, ts.s_w3);
        else
          gather_field3<kG3Edge, CKPT, kPutF32>(a, a.in, ld, lc, em[cb], nullptr, xrow, s_jrow, ts.s_w3);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    cscale[cb] = 1.0f;
    // First cell of the block (one 32-bit division per block) and the lane's
    // cell.  A block past the end of the lattice (in a ragged last tile)
    // takes the tile's first cell with every lane invalid.
    const int cbx = c0 + 32 * cb;
    const bool inside = (int64_t)cbx < g.C;
    const int base = inside ? cbx : c0;
    const int y0 = base / g.nx, x0 = base - y0 * g.nx;
    LaneCell lc = lane_cell(g, base, x0, y0, col);
    lc.valid = lc.valid && active && inside;
    lcs[cb] = lc;
    // per-cell coefficients, loaded now so that their latency is off the
    // epilogue's path (invalid lanes read the block's first cell)
    al[cb] = a.alpha[lc.c];
    be[cb] = a.beta[lc.c];
    em[cb] = a.emis[lc.c];
    if constexpr (MIX) {
      // (a batched channel without a mixture has nmix = 0 and no fractions)
      f0[cb] = a.nmix > 0 ? a.frac[lc.c] : 0.0f;
      float fs = f0[cb];
      for (int j = 1; j < a.nmix; ++j) fs += a.frac[(int64_t)j * g.C + lc.c];
      fr[cb] = 1.0f - fs;
    }
    // (a batched channel without dichroic absorption has no factors: xi = 0
    // makes them exactly 1)
    if constexpr (DICH) xi[cb] = a.dich_xi != nullptr ? a.dich_xi[lc.c] : 0.0f;
    // A block is interior when every tap of every cell lies inside the lattice
    // (taps reach at most two cells either way); then no wrap or ghost is needed.
    const int c_last = (int)((base + 32 < g.C ? (int64_t)base + 32 : g.C) - 1);
    const int ty1 = c_last / g.nx, tx1 = c_last - ty1 * g.nx;
    const bool interior = ty1 == y0 && y0 >= 2 && y0 <= g.ny - 3 && x0 >= 2 && tx1 <= g.nx - 3;
    inter[cb] = interior;
    if constexpr (XSPLIT) {
      // each combined group goes straight to the high and low tiles
      char *brow = s_b + (32 * cb + col) * L.strideB + rbase * 2;
      if (interior)
        gather_field<false, GATHER, true, true, CKPT, kPutSplit, DICH>(a, a.in, g, ld, lc, em[cb], nullptr, brow,
                                                                         s_jrow, L.tileB, xi[DICH ? cb : 0], wdir);
      else
        gather_field<false, GATHER, false, true, CKPT, kPutSplit, DICH>(a, a.in, g, ld, lc, em[cb], nullptr, brow,
                                                                          s_jrow, L.tileB, xi[DICH ? cb : 0], wdir);
    } else {
      // X (float32) goes to the X tile; the epilogue reads it back from there.
      char *xrow = s_x + (32 * cb + col) * L.strideX + rbase * 4;
      if (interior)
        gather_field<false, GATHER, true, true, CKPT, kPutF32, DICH>(a, a.in, g, ld, lc, em[cb], nullptr, xrow, s_jrow,
                                                                       0, xi[DICH ? cb : 0], wdir);
      else
        gather_field<false, GATHER, false, true, CKPT, kPutF32, DICH>(a, a.in, g, ld, lc, em[cb], nullptr, xrow,
                                                                        s_jrow, 0, xi[DICH ? cb : 0], wdir);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  }
  if constexpr (ADJ) {
    if constexpr (PREC == P_F32) {
      // the float32 B tile is mu itself: gathered straight into it
      char *murow = s_b + col * L.strideB + rbase * 4;
      if (inter[0])
        gather_field<true, true, true, false, false, kPutF32>(a, a.lam_next, g, ld, lcs[0], 0.0f, nullptr, murow,
                                                                s_jrow);
      else
        gather_field<true, true, false, false, false, kPutF32>(a, a.lam_next, g, ld, lcs[0], 0.0f, nullptr, murow,
                                                                 s_jrow);
    } else if constexpr (MUSPLIT) {
      char *murow = s_b + col * L.strideB + rbase * 2;
      if (inter[0])
        gather_field<true, true, true, false, false, kPutSplit>(a, a.lam_next, g, ld, lcs[0], 0.0f, nullptr, murow,
                                                                  s_jrow, L.tileB);
      else
        gather_field<true, true, false, false, false, kPutSplit>(a, a.lam_next, g, ld, lcs[0], 0.0f, nullptr, murow,
                                                                   s_jrow, L.tileB);
    } else {
      if (inter[0])
        gather_field<true, true, true, false, false, kPutReg>(a, a.lam_next, g, ld, lcs[0], 0.0f, mv, nullptr, s_jrow);
      else
        gather_field<true, true, false, false, false, kPutReg>(a, a.lam_next, g, ld, lcs[0], 0.0f, mv, nullptr, s_jrow);
    }
  }

  // ---- 3a. first A fragments in flight ---------------------------------------
  // A is the same for every tile; an L2 round trip for one K step is several
  // times longer than that step's MFMAs, so a ring of kRing steps is kept in
  // flight, started here to overlap the B conversion and the barrier.
  constexpr int kStep = PREC == P_F32 ? 8 : 16;
  // the bf16 contractions hold A (the collision matrix) as a bf16 high part
  // plus a bf16 low part: a single bf16 rounding of M shifts the
  // polarisation rows coherently at every step
  constexpr bool ALO = PREC == P_BF16 || PREC == P_BF16X3;
  const int nk = (tr.khi - tr.klo) / kStep;
  const uint4 *A = a.frag + lane;
  const uint4 *Alo = a.frag_lo + lane;
  uint4 ring[kRing], ring_lo[ALO ? kRing : 1];
#pragma unroll
  for (int j = 0; j < kRing; ++j) {
    ring[j] = A[frag_rec(tr, j, nk)];
    if (ALO) ring_lo[j] = Alo[frag_rec(tr, j, nk)];
  }

  // ---- 2. B operand: the contraction input in its precision ------------------
  // forward: X, adjoint: mu (both already in place for float32; X also for the
  // split tiles, mu for the bf16 / bf16x3 adjoint).
  if constexpr (!XSPLIT && !MUSPLIT) {
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
    if (PREC != P_F32) {
      char *xrow = s_x + (32 * cb + col) * L.strideX + rbase * 4;
      float v[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 x4;
        if constexpr (ADJ)
          x4 = f32x4{mv[4 * q], mv[4 * q + 1], mv[4 * q + 2], mv[4 * q + 3]};
        else
          x4 = *reinterpret_cast<const f32x4 *>(xrow + 32 * q);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * q + j] = x4[j];
      }
      // per-cell power-of-two scale for fp16 operands (max over all rows)
      if (PREC == P_F16) cscale[0] = f16_cell_scale(v, s_red, wg, W, col, h);
      char *brow = s_b + (32 * cb + col) * L.strideB;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r0 = rbase + q * 8;
        if (PREC == P_F32) {
          *reinterpret_cast<f32x4 *>(brow + r0 * 4) = f32x4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
        } else if (PREC == P_BF16 || PREC == P_BF16X3) {
          bf16x4 hv;
#pragma unroll
          for (int j = 0; j < 4; ++j) hv[j] = static_cast<__bf16>(v[4 * q + j]);
          *reinterpret_cast<bf16x4 *>(brow + r0 * 2) = hv;
          if (PREC == P_BF16X3) {
            bf16x4 lo;
#pragma unroll
            for (int j = 0; j < 4; ++j) lo[j] = static_cast<__bf16>(v[4 * q + j] - static_cast<float>(hv[j]));
            *reinterpret_cast<bf16x4 *>(brow + L.tileB + r0 * 2) = lo;
          }
        } else {
          f16x4 hv;
#pragma unroll
          for (int j = 0; j < 4; ++j) hv[j] = static_cast<_Float16>(v[4 * q + j] * cscale[0]);
          *reinterpret_cast<f16x4 *>(brow + r0 * 2) = hv;
        }
      }
    }
    }
  }
  __syncthreads();

  // ---- 3. matrix-core contraction over the tile's K range ------------------
  // Steps are taken in groups of kRing; steps past nk multiply the zero block
  // with the last valid B row (finite), adding nothing.  Every A fragment
  // serves the NB column blocks.
  f32x16 acc[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) acc[cb] = f32x16{0};
  // One contraction over the B tile: acc[cb] += A B for the tile's K range,
  // A from the fragment table Ap (and its low parts Alop for bf16 and
  // bf16x3), ring rg / rgl already holding its first kRing steps.
  auto contract = [&](const uint4 *Ap, const uint4 *Alop, const TileRange &trr, int nkk, uint4 (&rg)[kRing],
                      uint4 (&rgl)[ALO ? kRing : 1], f32x16 (&ac)[NB]) {
    const int nsteps = (nkk + kRing - 1) / kRing * kRing;
    // B fragments (16 bytes per lane per column block; bf16x3 also the low
    // part) are read from LDS one step ahead, so that their latency overlaps
    // the previous step's matrix-core work instead of preceding this step's
    constexpr int kLo = PREC == P_BF16X3 ? 2 : 1;
    auto bfrag = [&](int cb, int s, int part) -> uint4 {
      const int kb = trr.klo + kStep * min(s, nkk - 1);
      const char *bcell = s_b + (32 * cb + col) * L.strideB;
      const char *p = PREC == P_F32 ? bcell + (kb + 4 * h) * 4 : bcell + (kb + 8 * h) * 2 + part * L.tileB;
      return *reinterpret_cast<const uint4 *>(p);
    };
    uint4 bcur[NB][kLo];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int u = 0; u < kLo; ++u) bcur[cb][u] = bfrag(cb, 0, u);
    for (int s0 = 0; s0 < nsteps; s0 += kRing) {
#pragma unroll
      for (int j = 0; j < kRing; ++j) {
        const int s = s0 + j;
        const uint4 araw = rg[j], araw_lo = rgl[ALO ? j : 0];
        if constexpr (kRing == 1) {
          // a single slot: refill at once, so the load overlaps this step
          rg[j] = Ap[frag_rec(trr, s + kRing, nkk)];
          if (ALO) rgl[j] = Alop[frag_rec(trr, s + kRing, nkk)];
        }
        uint4 bnext[NB][kLo];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int u = 0; u < kLo; ++u) bnext[cb][u] = bfrag(cb, s + 1, u);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          if (PREC == P_F32) {
            const f32x4 av = __builtin_bit_cast(f32x4, araw);
            const f32x4 bv = __builtin_bit_cast(f32x4, bcur[cb][0]);
            ac[cb] = mfma_step_f32(av[0], bv[0], ac[cb]);
            ac[cb] = mfma_step_f32(av[1], bv[1], ac[cb]);
            ac[cb] = mfma_step_f32(av[2], bv[2], ac[cb]);
            ac[cb] = mfma_step_f32(av[3], bv[3], ac[cb]);
          } else if (PREC == P_F16) {
            const f16x8 av = __builtin_bit_cast(f16x8, araw);
            const f16x8 bv = __builtin_bit_cast(f16x8, bcur[cb][0]);
            ac[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, ac[cb], 0, 0, 0);
          } else {
            const bf16x8 av = __builtin_bit_cast(bf16x8, araw);
            const bf16x8 bv = __builtin_bit_cast(bf16x8, bcur[cb][0]);
            // the low part of A, then (bf16x3) the low part of B: the
            // leading products of (A_hi + A_lo)(B_hi + B_lo), smallest first
            const bf16x8 alo = __builtin_bit_cast(bf16x8, araw_lo);
            ac[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bv, ac[cb], 0, 0, 0);
            if (PREC == P_BF16X3) {
              const bf16x8 blo = __builtin_bit_cast(bf16x8, bcur[cb][kLo - 1]);
              ac[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, blo, ac[cb], 0, 0, 0);
            }
            ac[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, ac[cb], 0, 0, 0);
          }
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int u = 0; u < kLo; ++u) bcur[cb][u] = bnext[cb][u];
        if constexpr (kRing > 1) {
          __builtin_amdgcn_sched_barrier(0);
          rg[j] = Ap[frag_rec(trr, s + kRing, nkk)];
          if (ALO) rgl[j] = Alop[frag_rec(trr, s + kRing, nkk)];
        }
      }
    }
  };
  contract(A, Alo, tr, nk, ring, ring_lo, acc);
  // phase mixture: (1 - sum_j f_j) M X + sum_j f_j M_j X, each further
  // product contracted from the same B tile into acc2 and added at its
  // fraction (all products carry the same scale, undone in the epilogue);
  // f = 0 leaves M X exact, a one-hot f gives M_j X exactly
  f32x16 acc2[MIX ? NB : 1];
  if constexpr (MIX) {
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[cb][i] *= fr[cb];
    // the fraction of component m is at hand (f0, then loaded one contraction ahead)
    float fm[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) fm[cb] = f0[cb];
    for (int m = 0; m < a.nmix; ++m) {
      float fn[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) fn[cb] = m + 1 < a.nmix ? a.frac[(int64_t)(m + 1) * g.C + lcs[cb].c] : 0.0f;
      const TileRange tr2 = a.tiles2[m * (g.Rpad / 32) + t];   // 32-row tiles
      const int nk2 = (tr2.khi - tr2.klo) / kStep;
      const uint4 *A2 = a.frag2 + m * a.frag2_stride + lane;
      const uint4 *A2lo = a.frag2_lo + m * a.frag2_stride + lane;
#pragma unroll
      for (int j = 0; j < kRing; ++j) {
        ring[j] = A2[frag_rec(tr2, j, nk2)];
        if (ALO) ring_lo[j] = A2lo[frag_rec(tr2, j, nk2)];
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc2[cb] = f32x16{0};
      contract(A2, A2lo, tr2, nk2, ring, ring_lo, acc2);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[cb][i] = fmaf(fm[cb], acc2[cb][i], acc[cb][i]);
        fm[cb] = fn[cb];
      }
    }
  }
  (void)acc2;

  // ---- 4. epilogue -------------------------------------------------------------
  float part[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) part[k] = 0.0f;
  (void)gpre;
  // With NTC, forward steps store the output state non-temporally where it
  // exceeds the last-level cache (a.nt_out).  The loop then exists twice;
  // the non-temporal copy writes through the output base plus an opaque
  // zero, so that the compiler cannot merge the two copies' identical
  // stores, which would drop the hint (an integer offset keeps the base a
  // global pointer).
  auto epilogue = [&](auto nt_tag) {
  constexpr bool NT = decltype(nt_tag)::value;
  int64_t zoff = 0;
  if constexpr (NT) asm volatile("" : "+s"(zoff));
  float *outb = a.out + zoff;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    if (!lcs[cb].valid) continue;
    const int c = lcs[cb].c;
    const float unscale = a.a_scale_inv / cscale[cb];
    const char *xrow = s_x + (32 * cb + col) * L.strideX + rbase * 4;
    const char *brow = s_b + (32 * cb + col) * L.strideB;
    (void)xrow;
    (void)brow;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (ld[q].d >= g.n) continue;
      const f32x4 jp = *reinterpret_cast<const f32x4 *>(s_jrow + 4 * ld[q].d);
      f32x4 xq;
      if constexpr (XSPLIT) {
        // X = high + low (the sum is exact in float32)
        const int r0 = rbase + q * 8;
        const bf16x4 hv = *reinterpret_cast<const bf16x4 *>(brow + r0 * 2);
        const bf16x4 lv = *reinterpret_cast<const bf16x4 *>(brow + L.tileB + r0 * 2);
#pragma unroll
        for (int j = 0; j < 4; ++j) xq[j] = static_cast<float>(hv[j]) + static_cast<float>(lv[j]);
      } else {
        xq = *reinterpret_cast<const f32x4 *>(xrow + 32 * q);
      }
      // adjoint: mu of these 4 rows (for float32 it is the B tile itself)
      f32x4 mu = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (ADJ) {
        if constexpr (PREC == P_F32) {
          mu = *reinterpret_cast<const f32x4 *>(brow + (rbase + q * 8) * 4);
        } else if constexpr (MUSPLIT) {
          // mu = high + low, exact in float32 (to 2^-18 of mu)
          const bf16x4 hv = *reinterpret_cast<const bf16x4 *>(brow + (rbase + q * 8) * 2);
          const bf16x4 lv = *reinterpret_cast<const bf16x4 *>(brow + L.tileB + (rbase + q * 8) * 2);
#pragma unroll
          for (int j = 0; j < 4; ++j) mu[j] = static_cast<float>(hv[j]) + static_cast<float>(lv[j]);
        } else {
          mu = f32x4{mv[4 * q], mv[4 * q + 1], mv[4 * q + 2], mv[4 * q + 3]};
        }
      }
      float kap[ADJ && DICH ? 4 : 1];   // adjoint with dichroic absorption: dLoss/dX_d
      (void)kap;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int i = 4 * q + s;
        const float prod = acc[cb][i] * unscale;
        float *o = outb + ld[q].off + (int64_t)s * g.C + c;
        if (!ADJ) {
          const float y = fmaf(be[cb], prod, fmaf(al[cb], xq[s], a.dt_post * em[cb] * jp[s]));
          if constexpr (NT)
            __builtin_nontemporal_store(y, o);
          else
            *o = y;
        } else {
          // lam = dLoss/dX_d (X_d = X without dichroic absorption)
          const float lam = fmaf(be[cb], prod, al[cb] * mu[s]);
          part[0] = fmaf(mu[s], xq[s], part[0]);
          part[1] = fmaf(prod, xq[s], part[1]);
          if constexpr (DICH) {
            kap[s] = lam;
          } else {
            *o = lam;
            part[2] = fmaf(fmaf(a.dt_pre, lam, a.dt_post * mu[s]), jp[s], part[2]);
          }
        }
      }
      if constexpr (ADJ && DICH) {
        // dichroic absorption: X_d = D X with D scaling I + Q by exp(-xi w)
        // and I - Q by exp(xi w), symmetric in (I, Q), so dLoss/dX = D kap;
        // <kap, dD/dxi X> = -w (kap_I X_d,Q + kap_Q X_d,I)
        const float wq = wdir[q];
        part[3] = fmaf(-wq, fmaf(kap[0], xq[1], kap[1] * xq[0]), part[3]);
        dich_factor(kap[0], kap[1], xi[cb] * wq);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a.out[ld[q].off + (int64_t)s * g.C + c] = kap[s];
          part[2] = fmaf(fmaf(a.dt_pre, kap[s], a.dt_post * mu[s]), jp[s], part[2]);
        }
      }
    }
  }
  };
  if constexpr (NTC && !ADJ) {
    if (a.nt_out)
      epilogue(BoolTag<true>{});
    else
      epilogue(BoolTag<false>{});
  } else {
    epilogue(BoolTag<false>{});
  }
  if (ADJ) {
    // per-cell sums over all rows: half-waves, then waves via LDS
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
      float v = part[k];
      v += __shfl_xor(v, 32);
      if (h == 0) s_red[(k * W + wg) * 32 + col] = v;
    }
    __syncthreads();
    // (the lane index is made opaque so that the entry's address is formed
    // again here rather than held in registers through the tile)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    for (int e = wg * 64 + ln, u = 0; e < NACC * 32; e += W * 64, ++u) {
      const int k = e / 32, cc = e - k * 32;
      const int64_t c = (int64_t)c0 + cc;
      if (active && c < g.C) {
        double s = 0.0;
        for (int ww = 0; ww < W; ++ww) s += (double)s_red[(k * W + ww) * 32 + cc];
        double *p = a.gacc + (int64_t)k * g.C + c;
        *p = (u == 0 ? gpre : *p) + s;
      }
    }
  }
  __syncthreads();
}

// Resident blocks per CU of kernel k at this block size and LDS (registers
// and LDS of that instantiation), remembered in memo (one per instantiation)
// for the last (threads, LDS) asked.
inline hipError_t resident_blocks(const void *k, int threads, int lds, std::atomic<uint64_t> &memo, int *occ) {
  const uint64_t key = ((uint64_t)threads << 32) | (uint64_t)(uint32_t)lds;
  const uint64_t m = memo.load(std::memory_order_relaxed);
  if (m != 0 && (m >> 8) == key) {
    *occ = (int)(m & 0xff);
    return hipSuccess;
  }
  int o = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k, threads, lds);
  if (e != hipSuccess) return e;
  if (o < 1) return hipErrorInvalidConfiguration;
  o = std::min(o, 255);
  memo.store((key << 8) | (uint64_t)o, std::memory_order_relaxed);
  *occ = o;
  return hipSuccess;
}

// A-fragment ring depth: 4 steps for blocks of up to 4 waves (2 for the
// adjoint of the split-A bf16 contractions, whose ring holds low parts too);
// for the larger blocks (n > 32) the register budget of 16 waves per CU
// leaves 2 steps for the fp16 forward contraction and 1 otherwise.
template <int PREC, bool ADJ, int MAXW, int NB>
constexpr int kFusedRing = MAXW <= 4 ? (((ADJ && (PREC == P_BF16 || PREC == P_BF16X3)) || (NB > 1 && PREC == P_BF16)) ? 2 : 4)
                                     : ((!ADJ && PREC == P_F16) ? 2 : 1);

// Waves per SIMD the register allocation must allow: 4 for the fp32 and bf16
// adjoint in blocks of up to 4 waves (the accumulator then lives in ordinary
// VGPRs, without spills), 3 for the 3-D gather and the forward steps with a
// phase mixture or dichroic absorption in such blocks, otherwise whatever
// the kernel needs.
template <int PREC, bool ADJ, int MAXW, bool G3 = false, int EXT = kExtNone>
constexpr int kMinWavesPerEU = (ADJ && MAXW <= 4 && (PREC == P_F32 || PREC == P_BF16)) ? 4
                               : ((G3 || (!ADJ && EXT != kExtNone)) && MAXW <= 4) ? 3 : 1;

template <int PREC, bool GATHER, bool ADJ, int MAXW, bool CKPT, int NB, int EXT, bool G3 = false>
__global__ void __launch_bounds__(64 * MAXW) __attribute__((amdgpu_waves_per_eu(kMinWavesPerEU<PREC, ADJ, MAXW, G3, EXT>)))
fused_kernel(StepArgs a, int64_t ntiles) {
  using T = PrecTraits<PREC>;
  extern __shared__ __align__(16) char smem[];
  const Geometry g = a.geo;
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int h = lane >> 5;
  const LdsLayout L = lds_layout(g.Rpad, T::esize, T::ntile, W, ADJ, PREC == P_F16, 1, NB,
                                 (ADJ && EXT == kExtDich) ? 4 : 3, G3, kXSplit<PREC, MAXW, NB>);
  float *s_jrow = reinterpret_cast<float *>(smem + L.jrow_off);
  for (int i = threadIdx.x; i < g.Rpad; i += blockDim.x) s_jrow[i] = a.jrow[i];
  float *s_w3 = reinterpret_cast<float *>(smem + L.w3_off);
  if constexpr (G3) {
    // tap weights of the Rpad / 4 directions (zero for padding directions)
    for (int i = threadIdx.x; i < 2 * g.Rpad; i += blockDim.x) s_w3[i] = (i >> 3) < g.n ? a.taps3[i >> 3].w[i & 7] : 0.0f;
    for (int i = threadIdx.x; i < 2 * g.Rpad; i += blockDim.x) s_w3[2 * g.Rpad + i] = a.ghost[i];
  }
  __syncthreads();
  const TileLds ts{smem + L.b_off, smem + L.x_off, reinterpret_cast<float *>(smem + L.red_off), s_jrow, s_w3};

  const int t = __builtin_amdgcn_readfirstlane(w);  // the 32-row tile this wave owns
  const TileRange tr = a.tiles[t];
  // the lane's 4 directions: element group q holds direction 8 t + 2 q + h
  LaneDir ldk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ldk[q] = G3 ? lane_dir3(a, 8 * t + 2 * q + h) : lane_dir(a, 8 * t + 2 * q + h);

  // XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs,
  // so block b serves a contiguous eighth of the lattice and the halo rows it
  // reads stay in its XCD's L2.
  const int G = gridDim.x;
  const int chunks = (G >= 8 && (G & 7) == 0) ? 8 : 1;
  const int per = G / chunks;
  const int64_t kq = blockIdx.x % chunks;
  const int64_t first = ntiles * kq / chunks + blockIdx.x / chunks;
  const int64_t last = ntiles * (kq + 1) / chunks;

  for (int64_t tile = first; tile < last; tile += per) {
    // The direction data does not change between tiles.  Making it opaque in
    // place at every tile keeps the compiler from hoisting what derives from
    // it (16 plane pointers per buffer, the emission rows) out of the loop,
    // which would not fit in VGPRs, without holding a second copy.
#pragma unroll
    for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(ldk[q].off), "+v"(ldk[q].td), "+v"(ldk[q].d));
    fused_tile<PREC, GATHER, ADJ, CKPT, kFusedRing<PREC, ADJ, MAXW, NB>, NB, EXT, G3, kXSplit<PREC, MAXW, NB>,
               kNtCopy<ADJ, MAXW, NB, EXT, G3>>(a, g, L, ts, tr, ldk, tile, true, t, t, W, lane);
  }
}

// ------------------------------------------------------------- spectral batch --
//
// One launch advances every channel of one class (the channels with the
// same padded row count, hence the same waves per tile W) by one step.  A
// block has BW waves, BW / W tile groups side by side; the work queue is the
// class's channels' tiles in channel order, a work item being one tile per
// tile group of the block; the blocks of an XCD take every per-th item of one
// contiguous eighth of the queue, so each block changes channel only as
// often as its eighth does.  On a change the block reloads the channel's
// descriptor (scalar loads), its emission rows into LDS and each lane's
// direction data.

template <int PREC, bool GATHER, bool ADJ, bool CKPT, int BW, int EXT = kExtNone>
__global__ void __launch_bounds__(64 * BW) batch_kernel(const BatchChan *__restrict__ chans, int nchan,
                                                        int64_t nitems, BatchSel sel) {
  using T = PrecTraits<PREC>;
  extern __shared__ __align__(16) char smem[];
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // XCD-aware order, as in the single-problem kernel: blocks are dispatched
  // round-robin over the 8 XCDs; the blocks of one XCD interleave over one
  // contiguous eighth of the queue, so neighbouring tiles (and the halo rows
  // they share) are processed together in that XCD's L2.
  const int G = gridDim.x;
  const int chunks = (G >= 8 && (G & 7) == 0) ? 8 : 1;
  const int per = G / chunks;
  const int64_t kq = blockIdx.x % chunks;
  const int64_t i0 = nitems * kq / chunks + blockIdx.x / chunks;
  const int64_t i1 = nitems * (kq + 1) / chunks;

  int ch = -1;
  int64_t next0 = 0;   // first item of the next channel
  int64_t item0 = 0, ntiles = 0;
  int W = 1, grp = 0, t = 0;
  StepArgs a{};
  Geometry g{};
  LdsLayout L{};
  TileLds ts{};
  TileRange tr{};
  LaneDir ld[4];
  for (int64_t it = i0; it < i1; it += per) {
    if (ch < 0 || it >= next0) {
      int c = ch < 0 ? 0 : ch;
      while (c + 1 < nchan && chans[c + 1].item0 <= it) ++c;
      ch = c;
      const BatchChan &bc = chans[c];
      next0 = c + 1 < nchan ? chans[c + 1].item0 : nitems;
      item0 = bc.item0;
      ntiles = bc.ntiles;
      a = bc.a;
      auto bufp = [&](int id, int slot) -> float * {
        return id < 0 ? nullptr : bc.buf[id] + (int64_t)slot * bc.state_elems;
      };
      a.in = bufp(sel.in, sel.in_slot);
      a.out = bufp(sel.out, sel.out_slot);
      a.s_out = bufp(sel.sout, sel.sout_slot);
      a.lam_next = bufp(sel.lam, sel.lam_slot);
      g = a.geo;
      W = g.Rpad / 32;
      grp = w / W;
      t = w - grp * W;
      L = lds_layout(g.Rpad, T::esize, T::ntile, W, ADJ, PREC == P_F16, bc.groups, 1,
                     (ADJ && EXT == kExtDich) ? 4 : 3);
      char *gb = smem + grp * L.group;
      float *s_jrow = reinterpret_cast<float *>(smem + L.jrow_off);
      ts = TileLds{gb + L.b_off, gb + L.x_off, reinterpret_cast<float *>(gb + L.red_off), s_jrow, nullptr};
      tr = a.tiles[t];
#pragma unroll
      for (int q = 0; q < 4; ++q) ld[q] = lane_dir(a, 8 * t + 2 * q + h);
      __syncthreads();   // the previous channel's last tile is done with the LDS
      for (int i = threadIdx.x; i < g.Rpad; i += blockDim.x) s_jrow[i] = a.jrow[i];
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(ld[q].off), "+v"(ld[q].td), "+v"(ld[q].d));
    const int64_t tile = (it - item0) * (BW / W) + grp;
    // EXT: the phase-mixture or dichroic tile, for runs with such a channel
    // (a channel without the extension passes through it exactly: nmix = 0,
    // or xi = 0)
    fused_tile<PREC, GATHER, ADJ, CKPT, kFusedRing<PREC, ADJ, 4, 1>, 1, EXT>(
        a, g, L, ts, tr, ld, tile, tile < ntiles, t, t, W, lane);
  }
}

size_t batch_lds_bytes_impl(int Rpad, int prec, bool adjoint, int bw, bool dich) {
  const int W = Rpad / 32;
  if (W < 1 || W > kBatchWaves || bw < W || bw > kBatchWaves || bw % W != 0) return (size_t)-1;
  const int esize = prec == P_F32 ? 4 : 2;
  const int ntile = prec == P_BF16X3 ? 2 : 1;
  return (size_t)lds_layout(Rpad, esize, ntile, W, adjoint, prec == P_F16, bw / W, 1, (adjoint && dich) ? 4 : 3)
      .total;
}

// Occupancy of one batch instantiation; prepare_batch fills the memo before
// any launch, so a launch under stream capture makes no runtime query.
template <int PREC, bool GATHER, bool ADJ, bool CKPT, int BW, int EXT>
hipError_t batch_blocks_per_cu(int lds_bytes, int *occ) {
  static std::atomic<uint64_t> memo{0};
  return resident_blocks((const void *)batch_kernel<PREC, GATHER, ADJ, CKPT, BW, EXT>, 64 * BW, lds_bytes, memo,
                         occ);
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT, int BW, int EXT>
hipError_t prepare_batch_k(int lds_bytes, int *occ) {
  auto k = batch_kernel<PREC, GATHER, ADJ, CKPT, BW, EXT>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  int o = 0;
  e = batch_blocks_per_cu<PREC, GATHER, ADJ, CKPT, BW, EXT>(lds_bytes, &o);
  if (e != hipSuccess) return e;
  *occ = std::min(*occ, o);
  return hipSuccess;
}

template <int PREC, int BW, int EXT>
hipError_t prepare_batch_m(int lds_bytes, int *occ) {
  hipError_t e;
  if ((e = prepare_batch_k<PREC, false, false, false, BW, EXT>(lds_bytes, occ)) != hipSuccess) return e;
  if ((e = prepare_batch_k<PREC, true, false, false, BW, EXT>(lds_bytes, occ)) != hipSuccess) return e;
  if ((e = prepare_batch_k<PREC, true, false, true, BW, EXT>(lds_bytes, occ)) != hipSuccess) return e;
  if ((e = prepare_batch_k<PREC, false, true, false, BW, EXT>(lds_bytes, occ)) != hipSuccess) return e;
  return prepare_batch_k<PREC, true, true, false, BW, EXT>(lds_bytes, occ);
}

// blocks per CU: those of the instantiations without extensions (the
// phase-mixture and dichroic ones are prepared too, and size their own grids
// at launch)
template <int PREC, int BW>
hipError_t prepare_batch_p(int lds_bytes, int *occ) {
  hipError_t e = prepare_batch_m<PREC, BW, kExtNone>(lds_bytes, occ);
  if (e != hipSuccess) return e;
  int ext_occ = 1 << 20;
  if ((e = prepare_batch_m<PREC, BW, kExtMix>(lds_bytes, &ext_occ)) != hipSuccess) return e;
  return prepare_batch_m<PREC, BW, kExtDich>(lds_bytes, &ext_occ);
}

template <int PREC>
hipError_t prepare_batch_w(int bw, int lds_bytes, int *occ) {
  switch (bw) {
    case 1: return prepare_batch_p<PREC, 1>(lds_bytes, occ);
    case 2: return prepare_batch_p<PREC, 2>(lds_bytes, occ);
    case 4: return prepare_batch_p<PREC, 4>(lds_bytes, occ);
    case 8: return prepare_batch_p<PREC, 8>(lds_bytes, occ);
  }
  return hipErrorInvalidValue;
}

hipError_t prepare_batch_impl(int prec, int bw, int lds_bytes, int *blocks_per_cu) {
  int occ = 1 << 20;
  hipError_t e = hipErrorInvalidValue;
  if (prec == P_F32) e = prepare_batch_w<P_F32>(bw, lds_bytes, &occ);
  if (prec == P_BF16) e = prepare_batch_w<P_BF16>(bw, lds_bytes, &occ);
  if (prec == P_F16) e = prepare_batch_w<P_F16>(bw, lds_bytes, &occ);
  if (prec == P_BF16X3) e = prepare_batch_w<P_BF16X3>(bw, lds_bytes, &occ);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  *blocks_per_cu = occ;
  return hipSuccess;
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT, int BW, int EXT>
hipError_t launch_batch_k(const BatchChan *d_chans, int nchan, int64_t nitems, const BatchSel &sel, int lds_bytes,
                          int cu_count, hipStream_t s) {
  auto k = batch_kernel<PREC, GATHER, ADJ, CKPT, BW, EXT>;
  // persistent grid sized by this instantiation's own occupancy
  int occ = 0;
  const hipError_t e = batch_blocks_per_cu<PREC, GATHER, ADJ, CKPT, BW, EXT>(lds_bytes, &occ);
  if (e != hipSuccess) return e;
  int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)cu_count * occ));
  if (grid >= 8) grid &= ~7LL;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * BW), lds_bytes, s, d_chans, nchan, nitems, sel);
  return hipGetLastError();
}

template <int PREC, int BW, int EXT>
hipError_t launch_batch_m(const BatchChan *d_chans, int nchan, int64_t nitems, bool adjoint, bool gather, bool ckpt,
                          const BatchSel &sel, int lds_bytes, int cu_count, hipStream_t s) {
  if (adjoint) {
    if (gather)
      return launch_batch_k<PREC, true, true, false, BW, EXT>(d_chans, nchan, nitems, sel, lds_bytes, cu_count, s);
    return launch_batch_k<PREC, false, true, false, BW, EXT>(d_chans, nchan, nitems, sel, lds_bytes, cu_count, s);
  }
  if (ckpt) return launch_batch_k<PREC, true, false, true, BW, EXT>(d_chans, nchan, nitems, sel, lds_bytes, cu_count, s);
  if (gather)
    return launch_batch_k<PREC, true, false, false, BW, EXT>(d_chans, nchan, nitems, sel, lds_bytes, cu_count, s);
  return launch_batch_k<PREC, false, false, false, BW, EXT>(d_chans, nchan, nitems, sel, lds_bytes, cu_count, s);
}

template <int PREC, int BW>
hipError_t launch_batch_p(const BatchChan *d_chans, int nchan, int64_t nitems, bool adjoint, bool gather, bool ckpt,
                          int ext, const BatchSel &sel, int lds_bytes, int cu_count, hipStream_t s) {
  if (ext == kExtMix)
    return launch_batch_m<PREC, BW, kExtMix>(d_chans, nchan, nitems, adjoint, gather, ckpt, sel, lds_bytes, cu_count, s);
  if (ext == kExtDich)
    return launch_batch_m<PREC, BW, kExtDich>(d_chans, nchan, nitems, adjoint, gather, ckpt, sel, lds_bytes, cu_count, s);
  if (ext != kExtNone) return hipErrorInvalidValue;
  return launch_batch_m<PREC, BW, kExtNone>(d_chans, nchan, nitems, adjoint, gather, ckpt, sel, lds_bytes, cu_count, s);
}

template <int PREC>
hipError_t launch_batch_w(int bw, const BatchChan *d_chans, int nchan, int64_t nitems, bool adjoint, bool gather,
                          bool ckpt, int ext, const BatchSel &sel, int lds_bytes, int cu_count, hipStream_t s) {
  switch (bw) {
    case 1: return launch_batch_p<PREC, 1>(d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case 2: return launch_batch_p<PREC, 2>(d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case 4: return launch_batch_p<PREC, 4>(d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case 8: return launch_batch_p<PREC, 8>(d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_step_impl(const BatchChan *d_chans, int nchan, int64_t nitems, int prec, int bw,
                                  bool adjoint, bool gather, bool ckpt, int ext, const BatchSel &sel,
                                  int lds_bytes, int cu_count, hipStream_t s) {
  if (ckpt && (adjoint || !gather)) return hipErrorInvalidValue;
  if (cu_count < 1 || nitems < 1) return hipErrorInvalidValue;
  switch (prec) {
    case P_F32:
      return launch_batch_w<P_F32>(bw, d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case P_BF16:
      return launch_batch_w<P_BF16>(bw, d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case P_F16:
      return launch_batch_w<P_F16>(bw, d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes, cu_count, s);
    case P_BF16X3:
      return launch_batch_w<P_BF16X3>(bw, d_chans, nchan, nitems, adjoint, gather, ckpt, ext, sel, lds_bytes,
                                      cu_count, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT, int MAXW, int NB, int EXT = kExtNone, bool G3 = false>
hipError_t launch_fused_k(const StepArgs &a, int W, hipStream_t s, int cu_count) {
  using T = PrecTraits<PREC>;
  const LdsLayout L = lds_layout(a.geo.Rpad, T::esize, T::ntile, W, ADJ, PREC == P_F16, 1, NB,
                                 (ADJ && EXT == kExtDich) ? 4 : 3, G3, kXSplit<PREC, MAXW, NB>);
  if (L.total > 160 * 1024) return hipErrorInvalidValue;
  // 3-D: whole tiles per row (ny3 nz rows)
  const int64_t ntiles = G3 ? (int64_t)((a.geo.nx + 32 * NB - 1) / (32 * NB)) * a.ny3 * a.nz
                            : (a.geo.C + 32 * NB - 1) / (32 * NB);
  if (G3 && (a.zblk < 1 || a.ny3 * a.nz != a.geo.ny || ntiles > INT32_MAX)) return hipErrorInvalidValue;
  // strip order: a.strip tiles wide for 64-cell tiles, half as many (at
  // least one) for 32-cell tiles (the widths measured fastest per tile size)
  StepArgs args = a;
  if (!G3 && args.strip > 0) args.strip = NB == 2 ? args.strip : std::max(1, args.strip / 2);
  if (ntiles > INT32_MAX) return hipErrorInvalidValue;
  auto k = fused_kernel<PREC, GATHER, ADJ, MAXW, CKPT, NB, EXT, G3>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
  if (e != hipSuccess) return e;
  // persistent grid: as many blocks as are resident at once, so that no block
  // starts after others finish
  static std::atomic<uint64_t> memo{0};
  int occ = 0;
  e = resident_blocks((const void *)k, 64 * W, L.total, memo, &occ);
  if (e != hipSuccess) return e;
  int64_t grid = std::min<int64_t>(ntiles, (int64_t)cu_count * occ);
  if (grid >= 8) grid &= ~7LL;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * W), L.total, s, args, ntiles);
  return hipGetLastError();
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT>
hipError_t launch_fused_t(const StepArgs &a, int W, hipStream_t s, int cu_count);

// The 3-D fused forward step (float32 contraction): the tiles of the plain
// forward step.
template <bool CKPT>
hipError_t launch_fused3_t(const StepArgs &a, int W, hipStream_t s, int cu_count) {
  if (a.frac != nullptr || a.dich_xi != nullptr || a.taps3 == nullptr) return hipErrorInvalidValue;
  if (W <= 4) return launch_fused_k<P_F32, true, false, CKPT, 4, 2, kExtNone, true>(a, W, s, cu_count);
  return launch_fused_k<P_F32, true, false, CKPT, 16, 2, kExtNone, true>(a, W, s, cu_count);
}

template <int PREC, bool GATHER, bool ADJ, bool CKPT>
hipError_t launch_fused_t(const StepArgs &a, int W, hipStream_t s, int cu_count) {
  if (a.frac != nullptr && a.dich_xi != nullptr) return hipErrorInvalidValue;
  if (a.frac != nullptr) {
    // phase mixture, forward and adjoint: 32-cell tiles (the adjoint's
    // second matrix is M2^T, passed in the same fields)
    if (a.frag2 == nullptr || a.tiles2 == nullptr || a.nmix < 1) return hipErrorInvalidValue;
    if (W <= 4) return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 1, kExtMix>(a, W, s, cu_count);
    return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 1, kExtMix>(a, W, s, cu_count);
  }
  if (a.dich_xi != nullptr) {
    // dichroic absorption: the adjoint on 32-cell tiles; forward steps on the
    // tiles of the plain step
    if constexpr (ADJ) {
      if (W <= 4) return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 1, kExtDich>(a, W, s, cu_count);
      return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 1, kExtDich>(a, W, s, cu_count);
    } else {
      if (W <= 4) {
        if constexpr (PREC == P_F32 || PREC == P_BF16)
          return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 2, kExtDich>(a, W, s, cu_count);
        return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 1, kExtDich>(a, W, s, cu_count);
      }
      if constexpr (PREC == P_F32 || PREC == P_BF16) {
        if (step_nb(W, PREC, ADJ) == 2) return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 2, kExtDich>(a, W, s, cu_count);
      }
      return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 1, kExtDich>(a, W, s, cu_count);
    }
    return hipErrorInvalidValue;
  }
  if (W <= 4) {
    if constexpr (!ADJ && (PREC == P_F32 || PREC == P_BF16))
      return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 2>(a, W, s, cu_count);
    return launch_fused_k<PREC, GATHER, ADJ, CKPT, 4, 1>(a, W, s, cu_count);
  }
  if constexpr (!ADJ && (PREC == P_F32 || PREC == P_BF16)) {
    if (step_nb(W, PREC, ADJ) == 2) return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 2>(a, W, s, cu_count);
  }
  return launch_fused_k<PREC, GATHER, ADJ, CKPT, 16, 1>(a, W, s, cu_count);
}

// The checkpointing variant only exists for the forward gather (the step that
// produces S_t).
template <bool ADJ>
hipError_t launch_fused(const StepArgs &a, int prec, bool gather, hipStream_t s, int cu_count) {
  const int W = a.geo.Rpad / 32;
  if (W < 1 || W > 16) return hipErrorInvalidValue;
  const bool ckpt = !ADJ && a.s_out != nullptr;
  if (ckpt && !gather) return hipErrorInvalidValue;
#define RT_DISPATCH(P)                                                                       \
  if (prec == P) {                                                                           \
    if (ckpt) return launch_fused_t<P, true, ADJ, !ADJ>(a, W, s, cu_count);                  \
    if (gather) return launch_fused_t<P, true, ADJ, false>(a, W, s, cu_count);               \
    return launch_fused_t<P, false, ADJ, false>(a, W, s, cu_count);                          \
  }
  RT_DISPATCH(P_F32)
  RT_DISPATCH(P_BF16)
  RT_DISPATCH(P_F16)
  RT_DISPATCH(P_BF16X3)
#undef RT_DISPATCH
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- plain path --

// S_out[p](x, y) = pull of S_in[p] (Eq. 34) for every plane p = blockIdx.y;
// cells on the grid-stride loop, branch-free taps, the edge path only for
// cells within two cells of the lattice border.
__global__ void __launch_bounds__(256) stream_kernel(StepArgs a, const float *__restrict__ in,
                                                     float *__restrict__ out) {
  const Geometry g = a.geo;
  const int p = blockIdx.y;
  const int d = p >> 2, s = p & 3;
  const LaneDir ld = lane_dir(a, d);
  const int64_t plane = ld.off + (int64_t)s * g.C;
  const int C = (int)g.C;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
    const int y = c / g.nx;
    const int x = c - y * g.nx;
    float v[4];
    if (x >= 2 && x <= g.nx - 3 && y >= 2 && y <= g.ny - 3) {
      const float *p0 = in + plane + c - ld.td;
      const float *p1 = p0 - g.nx;
      v[0] = p0[0];
      v[1] = p0[-1];
      v[2] = p1[0];
      v[3] = p1[-1];
    } else {
      const LaneCell lc{c, x, y, true};
      const float *tp[4];
      int stride[4];
      edge_taps<false>(a, in, g, ld, lc, tp, stride);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = tp[k][(int64_t)s * stride[k]];
    }
    out[plane + c] = tap_sum(ld, v);
  }
}

// The same pull for nx a multiple of 4 and 16-byte aligned fields.  Each
// plane is split into interior quads (4 consecutive cells of a row, rows
// [2, ny - 3], cells [4, nx - 5], every tap inside the lattice) and the
// border ring (the remaining 4 nx + 8 (ny - 4) cells); a block takes one
// kind only, so no wave mixes the two paths.  An interior quad reads each of
// its two source rows as two aligned 16-byte vectors: with nx = 0 mod 4 the
// misalignment of the first tap, SH = (-ox0 - 1) mod 4, is the same for
// every cell of a plane, so it is a template argument chosen per block.
// A thread takes one quad column in two consecutive interior rows.
// Blocks are dispatched round-robin over the 8 XCDs; the block index is
// remapped so that each XCD takes one contiguous run of rows, and the two
// output rows that read a source row mostly share an L2.  Same arithmetic
// as stream_kernel (tap_sum), hence the same bits.
struct QuadSplit {
  int nqi, nri;     // interior quads per row, interior rows (both 0 if none)
  int int_blocks;   // blocks per plane taking interior quads
  int nbord;        // border cells per plane
  int bpp;          // blocks per plane
};

// One output quad from its two source rows (e: row y - oy0, f: the row
// below it), each given as the 8 aligned floats that start SH + 1 floats
// before the first cell's (0,0) tap.
template <int SH>
__device__ __forceinline__ void quad_out(const LaneDir &ld, const f32x4 &e0, const f32x4 &e1, const f32x4 &f0,
                                         const f32x4 &f1, float *dst) {
  const float e[8] = {e0[0], e0[1], e0[2], e0[3], e1[0], e1[1], e1[2], e1[3]};
  const float f[8] = {f0[0], f0[1], f0[2], f0[3], f1[0], f1[1], f1[2], f1[3]};
  float r4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float v[4] = {e[SH + k + 1], e[SH + k], f[SH + k + 1], f[SH + k]};
    r4[k] = tap_sum(ld, v);
  }
  *reinterpret_cast<f32x4 *>(dst) = f32x4{r4[0], r4[1], r4[2], r4[3]};
}

// Interior quad qi covers the same 4 columns of output rows y and y + 1
// (y + 1 only while it is an interior row): three source rows serve both.
template <int SH>
__device__ __forceinline__ void stream_interior_quads(const Geometry &g, const LaneDir &ld, int64_t plane,
                                                      int qi, int nqi, const float *__restrict__ in,
                                                      float *__restrict__ out) {
  const int r = qi / nqi;
  const int y = 2 + 2 * r;
  const int c = y * g.nx + 4 + 4 * (qi - r * nqi);
  const float *b = in + plane + c - ld.td - 1 - SH;   // 16-byte aligned
  const bool two = y + 1 <= g.ny - 3;
  const f32x4 e0 = *reinterpret_cast<const f32x4 *>(b);
  const f32x4 e1 = *reinterpret_cast<const f32x4 *>(b + 4);
  const f32x4 f0 = *reinterpret_cast<const f32x4 *>(b - g.nx);
  const f32x4 f1 = *reinterpret_cast<const f32x4 *>(b - g.nx + 4);
  f32x4 h0 = e0, h1 = e1;
  if (two) {
    h0 = *reinterpret_cast<const f32x4 *>(b + g.nx);
    h1 = *reinterpret_cast<const f32x4 *>(b + g.nx + 4);
  }
  quad_out<SH>(ld, e0, e1, f0, f1, out + plane + c);
  if (two) quad_out<SH>(ld, h0, h1, e0, e1, out + plane + c + g.nx);
}

__global__ void __launch_bounds__(256) stream4_kernel(StepArgs a, QuadSplit qs, const float *__restrict__ in,
                                                      float *__restrict__ out) {
  const Geometry g = a.geo;
  const int nb = gridDim.x, b = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = b & 7;
  const int lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + (b >> 3);
  const int p = lb / qs.bpp, bx = lb - p * qs.bpp;
  const LaneDir ld = lane_dir(a, p >> 2);
  const int s = p & 3;
  const int64_t plane = ld.off + (int64_t)s * g.C;
  if (bx < qs.int_blocks) {
    const int qi = bx * 256 + (int)threadIdx.x;
    if (qi >= qs.nqi * ((qs.nri + 1) >> 1)) return;
    switch ((-ld.ox0 - 1) & 3) {
      case 0: stream_interior_quads<0>(g, ld, plane, qi, qs.nqi, in, out); break;
      case 1: stream_interior_quads<1>(g, ld, plane, qi, qs.nqi, in, out); break;
      case 2: stream_interior_quads<2>(g, ld, plane, qi, qs.nqi, in, out); break;
      default: stream_interior_quads<3>(g, ld, plane, qi, qs.nqi, in, out); break;
    }
    return;
  }
  const int k = (bx - qs.int_blocks) * 256 + (int)threadIdx.x;
  if (k >= qs.nbord) return;
  int x, y;
  if (qs.nqi == 0) {           // no interior: the ring is the whole plane
    y = k / g.nx;
    x = k - y * g.nx;
  } else if (k < 4 * g.nx) {   // rows 0, 1, ny - 2, ny - 1
    const int r = k / g.nx;
    x = k - r * g.nx;
    y = r < 2 ? r : g.ny - 4 + r;
  } else {                     // rows 2 .. ny - 3: cells 0..3 and nx - 4 .. nx - 1
    const int m = k - 4 * g.nx, i = m & 7;
    y = 2 + (m >> 3);
    x = i < 4 ? i : g.nx - 8 + i;
  }
  const LaneCell lc{y * g.nx + x, x, y, true};
  const float *tp[4];
  int stride[4];
  edge_taps<false>(a, in, g, ld, lc, tp, stride);
  float v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = tp[t][(int64_t)s * stride[t]];
  out[plane + lc.c] = tap_sum(ld, v);
}

// Y(c) = alpha X(c) + beta M X(c) + dt_post J(c), X = S + dt_pre J, on the
// vector ALUs (the float32 path without matrix cores).  A wave takes 64
// consecutive cells, one per lane, and a group of kValuRows consecutive
// output rows (blockIdx.y): the lane accumulates its cell's rows in
// registers while the matrix entries, the same for the whole wave, arrive
// through scalar loads from M^T (row k = input row 4 d_in + s_in, contiguous
// over the output rows), so that one scalar load serves several rows.  Each
// input value is loaded once per row group.
constexpr int kValuRows = 32;

// Dichroic absorption of one direction's X (plain path): I + Q and I - Q
// scaled by exp(-+x).
__device__ __forceinline__ void dich_apply(float &xI, float &xQ, float x) { dich_factor(xI, xQ, x); }

template <bool DICH, bool MIX>
__global__ void __launch_bounds__(256) collide_valu_kernel(StepArgs a, const float *__restrict__ MT,
                                                           const float *__restrict__ in,
                                                           float *__restrict__ out) {
  const Geometry g = a.geo;
  const int R = g.R;   // 4 n, a multiple of 4
  const int r0 = blockIdx.y * kValuRows;
  const int nr = min(kValuRows, R - r0);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = c < g.C;
  const int64_t cc = valid ? c : 0;
  const float al = a.alpha[cc], be = a.beta[cc], em = a.emis[cc];
  const float edt = a.dt_pre * em;
  const float xi = DICH ? a.dich_xi[cc] : 0.0f;
  float acc[kValuRows], acc2[MIX ? kValuRows : 1];
  (void)acc2;
#pragma unroll
  for (int r = 0; r < kValuRows; ++r) acc[r] = 0.0f;
  // ac[r] += M[r0 + r][k] x_k over k; mk = MT + k R + r0 holds M[r0 + r][k] at mk[r]
  auto accumulate_into = [&](const float *__restrict__ T, float *ac, int k, float x) {
    const float *mk = T + (int64_t)k * R + r0;
#pragma unroll
    for (int r = 0; r < kValuRows; r += 16) {
      if (r + 16 <= nr) {
        const f32x16u m = *reinterpret_cast<const f32x16u *>(mk + r);
#pragma unroll
        for (int i = 0; i < 16; ++i) ac[r + i] = fmaf(m[i], x, ac[r + i]);
      } else {
#pragma unroll
        for (int q = r; q < r + 16; q += 4) {
          if (q < nr) {
            const f32x4 m = *reinterpret_cast<const f32x4 *>(mk + q);
#pragma unroll
            for (int i = 0; i < 4; ++i) ac[q + i] = fmaf(m[i], x, ac[q + i]);
          }
        }
      }
    }
  };
  auto accumulate = [&](int k, float x) { accumulate_into(MT, acc, k, x); };
  if constexpr (MIX) {
    // phase mixture: acc = (1 - sum_j f_j) M X, then f_j M_j X added per
    // further matrix (its product in acc2; X read again for each)
    float fs = a.frac[cc];
    for (int j = 1; j < a.nmix; ++j) fs += a.frac[(int64_t)j * g.C + cc];
    for (int k = 0; k < R; ++k) accumulate(k, fmaf(edt, a.jrow[k], in[(int64_t)k * g.C + cc]));
    const float w0 = 1.0f - fs;
#pragma unroll
    for (int r = 0; r < kValuRows; ++r) acc[r] *= w0;
    for (int j = 0; j < a.nmix; ++j) {
      const float *MTj = a.MT2 + (int64_t)j * R * R;
      const float fj = a.frac[(int64_t)j * g.C + cc];
#pragma unroll
      for (int r = 0; r < kValuRows; ++r) acc2[r] = 0.0f;
      for (int k = 0; k < R; ++k) accumulate_into(MTj, acc2, k, fmaf(edt, a.jrow[k], in[(int64_t)k * g.C + cc]));
#pragma unroll
      for (int r = 0; r < kValuRows; ++r) acc[r] = fmaf(fj, acc2[r], acc[r]);
    }
  } else if constexpr (DICH) {
    // one direction (4 Stokes rows) at a time: its I and Q are combined
    for (int k = 0; k < R; k += 4) {
      float x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = fmaf(edt, a.jrow[k + j], in[(int64_t)(k + j) * g.C + cc]);
      dich_apply(x[0], x[1], xi * a.dich_w[k / 4]);
#pragma unroll
      for (int j = 0; j < 4; ++j) accumulate(k + j, x[j]);
    }
  } else {
    for (int k = 0; k < R; ++k) accumulate(k, fmaf(edt, a.jrow[k], in[(int64_t)k * g.C + cc]));
  }
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < kValuRows; r += 4) {
    if (r < nr) {
      float xo[4], jr[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        jr[j] = a.jrow[r0 + r + j];
        xo[j] = fmaf(edt, jr[j], in[(int64_t)(r0 + r + j) * g.C + c]);
      }
      if constexpr (DICH) dich_apply(xo[0], xo[1], xi * a.dich_w[(r0 + r) / 4]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        out[(int64_t)(r0 + r + j) * g.C + c] = fmaf(be, acc[r + j], fmaf(al, xo[j], a.dt_post * em * jr[j]));
      }
    }
  }
}

// Streaming on a 3-D lattice: out[4d + s](x, y, z) = sum over the 8 taps b of
// w_b in[4d + s](x - ox0 - bx, y - oy0 - by, z - oz0 - bz) (the pull of Eq. 34
// along each axis).  Periodic axes wrap; a tap still outside reads the ghost
// radiance of its face (z before y before x; zero for absorbing faces).
//
// Columns x in [4, nx - 5] (nx a multiple of 4: "quad columns") have every
// x tap inside the lattice.  There a thread produces 4 consecutive cells of
// kRowsQ rows of one plane over kZRun layers, sliding along z so that each
// layer step loads one new source layer of kRowsQ + 1 rows (two aligned
// 16-byte loads per row, or, for a row outside the lattice in y or z, its
// face's ghost value, uniform along the row).  The 8 end columns of every row
// take one thread per cell with the general tap rules.
constexpr int kZRun = 8;    // layers per quad-column thread
constexpr int kRowsQ = 2;   // rows per quad-column thread

struct Box3 {
  int on;          // quad columns exist (nx a multiple of 4, nx >= 12, aligned fields)
  int nqx;         // quads per row
  int nyp, nq;     // row groups (kRowsQ rows) per layer; quad-column threads per plane (kZRun layers each)
  int nbord;       // cells of the end columns (all cells when `on` is 0)
  int ib;          // blocks per plane taking quads
  int bpp;         // blocks per plane
};

// Loads one source layer zs (kRowsQ + 1 rows y - oy0 - 1 + {0 .. kRowsQ}) of a quad column:
// each row as the 8 aligned floats that start SH + 1 floats before the first
// cell's bx = 0 tap, or the ghost value of its face for a row outside the
// lattice in y or z.
template <int SH>
__device__ __forceinline__ void quad3_layer(const Stream3Args &g, const DirTaps3 &tp, const float *__restrict__ in,
                                            int64_t plane, int p, int x0, int y, int zs,
                                            float (&e)[kRowsQ + 1][8]) {
  const int64_t layer = (int64_t)g.ny * g.nx;
  const int zw = wrap_axis(zs, g.nz, g.per_z);
  const bool inz = (unsigned)zw < (unsigned)g.nz;
#pragma unroll
  for (int b = 0; b < kRowsQ + 1; ++b) {
    const int ys = wrap_axis(y - tp.oy0 + b - 1, g.ny, g.per_y);
    const bool iny = (unsigned)ys < (unsigned)g.ny;
    if (inz && iny) {
      const float *r = in + plane + zw * layer + (int64_t)ys * g.nx + x0 - tp.ox0 - 1 - SH;
      const f32x4 v0 = *reinterpret_cast<const f32x4 *>(r);
      const f32x4 v1 = *reinterpret_cast<const f32x4 *>(r + 4);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        e[b][k] = v0[k];
        e[b][k + 4] = v1[k];
      }
    } else {
      const float gv = g.ghost[(!inz ? (zw < 0 ? 4 : 5) : (ys < 0 ? 2 : 3)) * g.Rpad + p];
#pragma unroll
      for (int k = 0; k < 8; ++k) e[b][k] = gv;
    }
  }
}

// A quad column of kRowsQ rows (y, y + 1, ...; those below ny) over the
// layers z0 .. z1 - 1, sliding along z: output layer z reads source layers
// z - oz0 - 1 (bz = 1) and z - oz0 (bz = 0), so each step loads one new
// source layer (kRowsQ + 1 rows) and keeps the previous one.
template <int SH>
__device__ __forceinline__ void quad3_column(const Stream3Args &g, const DirTaps3 &tp, const float *__restrict__ in,
                                             int64_t plane, int p, int x0, int y, int z0, int z1,
                                             float *__restrict__ out) {
  const int64_t layer = (int64_t)g.ny * g.nx;
  float hi[kRowsQ + 1][8], lo[kRowsQ + 1][8];   // source layers z - oz0 (bz = 0) and z - oz0 - 1 (bz = 1)
  quad3_layer<SH>(g, tp, in, plane, p, x0, y, z0 - tp.oz0 - 1, lo);
  for (int z = z0; z < z1; ++z) {
    quad3_layer<SH>(g, tp, in, plane, p, x0, y, z - tp.oz0, hi);
#pragma unroll
    for (int j = 0; j < kRowsQ; ++j) {
      if (y + j >= g.ny) continue;
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int bz = 0; bz < 2; ++bz)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          const float *ev = bz ? lo[j - by + 1] : hi[j - by + 1];
          const float w0 = tp.w[4 * bz + 2 * by], w1 = tp.w[4 * bz + 2 * by + 1];
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] = fmaf(w1, ev[SH + k], fmaf(w0, ev[SH + k + 1], acc[k]));
        }
      *reinterpret_cast<f32x4 *>(out + plane + z * layer + (int64_t)(y + j) * g.nx + x0) =
          f32x4{acc[0], acc[1], acc[2], acc[3]};
    }
#pragma unroll
    for (int b = 0; b < kRowsQ + 1; ++b)
#pragma unroll
      for (int k = 0; k < 8; ++k) lo[b][k] = hi[b][k];
  }
}

// box.bpp blocks per plane p = 4 d + s: the first box.ib take quad columns,
// of quads, the rest one end-column cell per thread.  Blocks are dispatched
// round-robin over the 8 XCDs; the logical order is remapped so that each XCD
// takes a contiguous range, and the source rows that neighbouring blocks of a
// plane share stay in one XCD's L2.
__global__ void __launch_bounds__(256) stream3d_kernel(Stream3Args g, Box3 box, const float *__restrict__ in,
                                                       float *__restrict__ out) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, xcd = b & 7;
  const int lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + (b >> 3);
  const int p = lb / box.bpp, bx = lb - p * box.bpp;
  const DirTaps3 tp = g.taps[p >> 2];
  const int64_t plane = (int64_t)p * g.C;
  if (bx < box.ib) {
    const int q = bx * blockDim.x + threadIdx.x;
    if (q >= box.nq) return;
    const int qx = q % box.nqx;
    const int t = q / box.nqx;
    const int y = kRowsQ * (t % box.nyp);
    const int z0 = kZRun * (t / box.nyp);
    const int z1 = min(z0 + kZRun, g.nz);
    const int x0 = 4 + 4 * qx;
    switch ((-tp.ox0 - 1) & 3) {
      case 0: quad3_column<0>(g, tp, in, plane, p, x0, y, z0, z1, out); break;
      case 1: quad3_column<1>(g, tp, in, plane, p, x0, y, z0, z1, out); break;
      case 2: quad3_column<2>(g, tp, in, plane, p, x0, y, z0, z1, out); break;
      default: quad3_column<3>(g, tp, in, plane, p, x0, y, z0, z1, out); break;
    }
    return;
  }
  const int k = (bx - box.ib) * blockDim.x + threadIdx.x;
  if (k >= box.nbord) return;
  int x, y, z;
  if (box.on) {   // the 4 + 4 end cells of row r = z ny + y
    const int r = k >> 3, i = k & 7;
    x = i < 4 ? i : g.nx - 8 + i;
    y = r % g.ny;
    z = r / g.ny;
  } else {
    x = k % g.nx;
    const int t = k / g.nx;
    y = t % g.ny;
    z = t / g.ny;
  }
  float acc = 0.0f;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const float w = tp.w[b];
    if (w == 0.0f) continue;   // the same taps vanish for the whole direction
    const int xs = wrap_axis(x - tp.ox0 - (b & 1), g.nx, g.per_x);
    const int ys = wrap_axis(y - tp.oy0 - ((b >> 1) & 1), g.ny, g.per_y);
    const int zs = wrap_axis(z - tp.oz0 - (b >> 2), g.nz, g.per_z);
    const bool inside = (unsigned)xs < (unsigned)g.nx && (unsigned)ys < (unsigned)g.ny &&
                        (unsigned)zs < (unsigned)g.nz;
    const int f = (unsigned)zs >= (unsigned)g.nz ? (zs < 0 ? 4 : 5)
                  : ((unsigned)ys >= (unsigned)g.ny ? (ys < 0 ? 2 : 3) : (xs < 0 ? 0 : 1));
    const float v = inside ? in[plane + ((int64_t)zs * g.ny + ys) * g.nx + xs] : g.ghost[f * g.Rpad + p];
    acc = fmaf(w, v, acc);
  }
  out[plane + ((int64_t)z * g.ny + y) * g.nx + x] = acc;
}

// ------------------------------------------------------------- small kernels --

__global__ void coef_kernel(int64_t C, const float *__restrict__ tau, const float *__restrict__ alb,
                            const float *__restrict__ emis, float *tau_c, float *alb_c, float *emis_c,
                            float *alpha, float *beta, uint32_t flags, int *bad) {
  int nbad = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double t = tau[c], w = alb[c], e = emis[c];
    double al = 0.0, be = 0.0;
    bool ok = std::isfinite(t) && std::isfinite(w) && std::isfinite(e) && t >= 0.0 && w >= 0.0 &&
              w <= 1.0;
    if (ok) {
      const double tsca = w * t, tabs = (1.0 - w) * t;
      if (flags & RT_FUSED_TAYLOR) {
        al = 1.0 - t;
        be = tsca;
        ok = al >= 0.0;
      } else {
        const double aa = (flags & RT_ABS_TAYLOR) ? 1.0 - tabs : std::exp(-tabs);
        const double ss = (flags & RT_SCAT_EXP) ? std::exp(-tsca) : 1.0 - tsca;
        ok = aa >= 0.0 && ss >= 0.0;
        al = aa * ss;
        be = aa * (1.0 - ss);
      }
    }
    if (!ok) ++nbad;
    tau_c[c] = (float)t;
    alb_c[c] = (float)w;
    emis_c[c] = (float)e;
    alpha[c] = (float)al;
    beta[c] = (float)be;
  }
  if (nbad) atomicAdd(bad, nbad);
}

// Dichroic absorption per cell: xi = tau_abs * eta = (1 - albedo) tau eta
// (float64 arithmetic, stored in float32); counts |eta| >= 1 or non-finite
// eta into *bad.
__global__ void dich_xi_kernel(int64_t C, const float *__restrict__ tau, const float *__restrict__ alb,
                               const float *__restrict__ eta, float *xi, int *bad) {
  int nbad = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double e = eta[c];
    if (!(std::fabs(e) < 1.0)) ++nbad;
    xi[c] = (float)((1.0 - (double)alb[c]) * (double)tau[c] * e);
  }
  if (nbad) atomicAdd(bad, nbad);
}

__global__ void gradchain_kernel(int64_t C, const float *__restrict__ tau, const float *__restrict__ alb,
                                 uint32_t flags, const double *__restrict__ gacc, float *g_tau,
                                 float *g_alb, float *g_emis, const float *__restrict__ eta) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const double t = tau[c], w = alb[c];
    const double ga = gacc[c], gb = gacc[C + c], ge = gacc[2 * C + c];
    double dat, daw, dbt, dbw;
    if (flags & RT_FUSED_TAYLOR) {
      dat = -1.0; daw = 0.0; dbt = w; dbw = t;
    } else {
      const double tabs = (1.0 - w) * t, tsca = w * t;
      double aa, da_t, da_w, ss, ds_t, ds_w;
      if (flags & RT_ABS_TAYLOR) { aa = 1.0 - tabs; da_t = -(1.0 - w); da_w = t; }
      else { aa = std::exp(-tabs); da_t = -(1.0 - w) * aa; da_w = t * aa; }
      if (flags & RT_SCAT_EXP) { ss = std::exp(-tsca); ds_t = -w * ss; ds_w = -t * ss; }
      else { ss = 1.0 - tsca; ds_t = -w; ds_w = -t; }
      dat = da_t * ss + aa * ds_t;
      daw = da_w * ss + aa * ds_w;
      dbt = da_t * (1.0 - ss) - aa * ds_t;
      dbw = da_w * (1.0 - ss) - aa * ds_w;
    }
    // dichroic absorption: xi = (1 - albedo) tau eta, its sum in gacc[3 C + c]
    double gxt = 0.0, gxw = 0.0;
    if (eta) {
      const double gx = gacc[3 * C + c], e = eta[c];
      gxt = gx * (1.0 - w) * e;
      gxw = -gx * t * e;
    }
    if (g_tau) g_tau[c] = (float)(ga * dat + gb * dbt + gxt);
    if (g_alb) g_alb[c] = (float)(ga * daw + gb * dbw + gxw);
    if (g_emis) g_emis[c] = (float)ge;
  }
}

template <typename V>
__global__ void fill_kernel(V *p, int64_t count, V v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ int64_t edge_cell(const Geometry &g, int edge, int e) {
  if (edge == kEdgeYp) return (int64_t)(g.ny - 1) * g.nx + e;
  if (edge == kEdgeYm) return e;
  if (edge == kEdgeXp) return (int64_t)e * g.nx + (g.nx - 1);
  return (int64_t)e * g.nx;
}

__global__ void readout_kernel(Geometry g, const float *__restrict__ S, int edge,
                               const int32_t *__restrict__ dirs, int nout, int nedge, float *out) {
  const int64_t total = (int64_t)nedge * nout * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i & 3);
    const int k = (int)((i >> 2) % nout);
    const int e = (int)((i >> 2) / nout);
    out[i] = S[(int64_t)(4 * dirs[k] + s) * g.C + edge_cell(g, edge, e)];
  }
}

__global__ void readout_adjoint_kernel(Geometry g, int edge, const int32_t *__restrict__ dirs, int nout,
                                       int nedge, const float *__restrict__ gout, float *lam) {
  const int64_t total = (int64_t)nedge * nout * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i & 3);
    const int k = (int)((i >> 2) % nout);
    const int e = (int)((i >> 2) / nout);
    lam[(int64_t)(4 * dirs[k] + s) * g.C + edge_cell(g, edge, e)] = gout[i];
  }
}

// Face readouts of a 3-D lattice: face cell e = a + na b lies at
// base + a sa + b sb (FaceMap), out[e][k][s] = S[4 dirs[k] + s](cell).
__global__ void readout_face_kernel(int64_t C, FaceMap f, const float *__restrict__ S,
                                    const int32_t *__restrict__ dirs, int nout, float *out) {
  const int64_t total = (int64_t)f.count * nout * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i & 3);
    const int k = (int)((i >> 2) % nout);
    const int e = (int)((i >> 2) / nout);
    const int64_t cell = f.base + (int64_t)(e % f.na) * f.sa + (int64_t)(e / f.na) * f.sb;
    out[i] = S[(int64_t)(4 * dirs[k] + s) * C + cell];
  }
}

__global__ void readout_face_adjoint_kernel(int64_t C, FaceMap f, const int32_t *__restrict__ dirs, int nout,
                                            const float *__restrict__ gout, float *lam) {
  const int64_t total = (int64_t)f.count * nout * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i & 3);
    const int k = (int)((i >> 2) % nout);
    const int e = (int)((i >> 2) / nout);
    const int64_t cell = f.base + (int64_t)(e % f.na) * f.sa + (int64_t)(e / f.na) * f.sb;
    lam[(int64_t)(4 * dirs[k] + s) * C + cell] = gout[i];
  }
}

constexpr int kSumThreads = 256;

// Partial float64 sums of the I, Q, U, V planes: block b covers a fixed range
// of cells for every direction, so the reduction order is fixed.
__global__ void __launch_bounds__(kSumThreads) sums_kernel(Geometry g, const float *__restrict__ S,
                                                           double *partial) {
  __shared__ double red[4][kSumThreads];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.C;
       c += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < g.n; ++d)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] += (double)S[(int64_t)(4 * d + s) * g.C + c];
#pragma unroll
  for (int s = 0; s < 4; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int off = kSumThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int s = 0; s < 4; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void sums_final_kernel(const double *__restrict__ partial, int npart, double *result) {
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int b = 0; b < npart; ++b) s += partial[b * 4 + threadIdx.x];
    result[threadIdx.x] = s;
  }
}

__global__ void maps_kernel(Geometry g, const float *__restrict__ S, float *I_mean, float *dop_mean) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.C;
       c += (int64_t)gridDim.x * blockDim.x) {
    float si = 0.f, sd = 0.f;
    for (int d = 0; d < g.n; ++d) {
      const float I = S[(int64_t)(4 * d) * g.C + c];
      const float Q = S[(int64_t)(4 * d + 1) * g.C + c];
      const float U = S[(int64_t)(4 * d + 2) * g.C + c];
      const float V = S[(int64_t)(4 * d + 3) * g.C + c];
      si += I;
      if (I > 0.f) sd += sqrtf(Q * Q + U * U + V * V) / I;
    }
    I_mean[c] = si / g.n;
    dop_mean[c] = sd / g.n;
  }
}

inline unsigned grid_for(int64_t work, int threads, int64_t cap = 4096) {
  int64_t b = (work + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

size_t batch_lds_bytes(int Rpad, int prec, bool adjoint, int bw, bool dich) {
  return batch_lds_bytes_impl(Rpad, prec, adjoint, bw, dich);
}

hipError_t prepare_batch(int prec, int bw, int lds_bytes, int *blocks_per_cu) {
  return prepare_batch_impl(prec, bw, lds_bytes, blocks_per_cu);
}

hipError_t launch_batch_step(const BatchChan *d_chans, int nchan, int64_t nitems, int prec, int bw, bool adjoint,
                             bool gather, bool ckpt, int ext, const BatchSel &sel, int lds_bytes, int cu_count,
                             hipStream_t s) {
  return launch_batch_step_impl(d_chans, nchan, nitems, prec, bw, adjoint, gather, ckpt, ext, sel, lds_bytes,
                                cu_count, s);
}

size_t step_lds_bytes(const Geometry &g, int prec, bool adjoint, bool dich, bool three_d) {
  if (g.Rpad / 32 > 16) return (size_t)-1;
  const int esize = prec == P_F32 ? 4 : 2;
  const int ntile = prec == P_BF16X3 ? 2 : 1;
  const int W = g.Rpad / 32;
  const int nb = step_nb(W, prec, adjoint);
  const LdsLayout L = lds_layout(g.Rpad, esize, ntile, W, adjoint, prec == P_F16, 1, nb, adjoint && dich ? 4 : 3,
                                 three_d && !adjoint, nb > 1 && prec == P_BF16 && W > 4);
  return (size_t)L.total;
}

hipError_t launch_step3_mfma(const StepArgs &a, int prec, hipStream_t s, int cu_count) {
  const int W = a.geo.Rpad / 32;
  if (W < 1 || W > 16 || prec != P_F32) return hipErrorInvalidValue;
  if (a.s_out != nullptr) return launch_fused3_t<true>(a, W, s, cu_count);
  return launch_fused3_t<false>(a, W, s, cu_count);
}

hipError_t launch_step_mfma(const StepArgs &a, int prec, bool gather, hipStream_t s, int cu_count) {
  return launch_fused<false>(a, prec, gather, s, cu_count);
}

hipError_t launch_adjoint_mfma(const StepArgs &a, int prec, bool gather, hipStream_t s, int cu_count) {
  return launch_fused<true>(a, prec, gather, s, cu_count);
}

hipError_t launch_stream(const StepArgs &a, const float *in, float *out, hipStream_t s) {
  const bool quads = a.geo.nx % 4 == 0 && ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  if (quads) {
    QuadSplit qs;
    qs.nqi = std::max(0, a.geo.nx / 4 - 2);
    qs.nri = std::max(0, a.geo.ny - 4);
    if (qs.nqi == 0 || qs.nri == 0) qs.nqi = qs.nri = 0;
    const int64_t nint = (int64_t)qs.nqi * qs.nri;
    qs.nbord = (int)(a.geo.C - 4 * nint);
    qs.int_blocks = (int)(((int64_t)qs.nqi * ((qs.nri + 1) / 2) + 255) / 256);   // two rows per thread
    qs.bpp = qs.int_blocks + (qs.nbord + 255) / 256;
    const int64_t blocks = (int64_t)qs.bpp * 4 * a.geo.n;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream4_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, qs, in, out);
  } else {
    dim3 grid(grid_for(a.geo.C, 256, 1024), 4 * a.geo.n);
    hipLaunchKernelGGL(stream_kernel, grid, dim3(256), 0, s, a, in, out);
  }
  return hipGetLastError();
}

hipError_t launch_collide_valu(const StepArgs &a, const float *MT, const float *in, float *out,
                               hipStream_t s) {
  const dim3 grid((unsigned)((a.geo.C + 255) / 256), (unsigned)((a.geo.R + kValuRows - 1) / kValuRows));
  if (a.dich_xi != nullptr && a.frac != nullptr) return hipErrorInvalidValue;
  if (a.dich_xi != nullptr)
    hipLaunchKernelGGL((collide_valu_kernel<true, false>), grid, dim3(256), 0, s, a, MT, in, out);
  else if (a.frac != nullptr) {
    if (a.MT2 == nullptr || a.nmix < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((collide_valu_kernel<false, true>), grid, dim3(256), 0, s, a, MT, in, out);
  }
  else
    hipLaunchKernelGGL((collide_valu_kernel<false, false>), grid, dim3(256), 0, s, a, MT, in, out);
  return hipGetLastError();
}

hipError_t launch_stream3d(const Stream3Args &a, const float *in, float *out, hipStream_t s) {
  if (a.n < 1 || 4 * a.n > 65535 || a.C < 1) return hipErrorInvalidValue;
  Box3 box{0, 0, 0, 0, (int)a.C, 0, 0};
  const bool aligned = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  if (aligned && a.nx % 4 == 0 && a.nx >= 12) {
    box.on = 1;
    box.nqx = a.nx / 4 - 2;
    box.nyp = (a.ny + kRowsQ - 1) / kRowsQ;
    box.nq = box.nqx * box.nyp * ((a.nz + kZRun - 1) / kZRun);
    box.nbord = 8 * a.ny * a.nz;
    box.ib = (box.nq + 255) / 256;
  }
  box.bpp = box.ib + (box.nbord + 255) / 256;
  const int64_t blocks = (int64_t)box.bpp * 4 * a.n;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream3d_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, box, in, out);
  return hipGetLastError();
}

hipError_t launch_coef(int64_t C, const float *tau, const float *alb, const float *emis, float *tau_c,
                       float *alb_c, float *emis_c, float *alpha, float *beta, uint32_t flags, int *bad,
                       hipStream_t s) {
  hipLaunchKernelGGL(coef_kernel, dim3(grid_for(C, 256)), dim3(256), 0, s, C, tau, alb, emis, tau_c,
                     alb_c, emis_c, alpha, beta, flags, bad);
  return hipGetLastError();
}

hipError_t launch_dich_xi(int64_t C, const float *tau, const float *alb, const float *eta, float *xi, int *bad,
                          hipStream_t s) {
  hipLaunchKernelGGL(dich_xi_kernel, dim3(grid_for(C, 256)), dim3(256), 0, s, C, tau, alb, eta, xi, bad);
  return hipGetLastError();
}

hipError_t launch_gradchain(int64_t C, const float *tau, const float *alb, uint32_t flags,
                            const double *gacc, float *g_tau, float *g_alb, float *g_emis,
                            hipStream_t s, const float *eta) {
  hipLaunchKernelGGL(gradchain_kernel, dim3(grid_for(C, 256)), dim3(256), 0, s, C, tau, alb, flags,
                     gacc, g_tau, g_alb, g_emis, eta);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t count, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

static int edge_len(const Geometry &g, int edge) { return edge >= 2 ? g.nx : g.ny; }

hipError_t launch_readout(const Geometry &g, const float *S, int edge, const int32_t *dirs, int nout,
                          float *out, hipStream_t s) {
  const int ne = edge_len(g, edge);
  const int64_t total = (int64_t)ne * nout * 4;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(readout_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g, S, edge, dirs, nout,
                     ne, out);
  return hipGetLastError();
}

hipError_t launch_readout_adjoint(const Geometry &g, int edge, const int32_t *dirs, int nout,
                                  const float *gout, float *lam, hipStream_t s) {
  const int ne = edge_len(g, edge);
  const int64_t total = (int64_t)ne * nout * 4;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(readout_adjoint_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, g, edge, dirs,
                     nout, ne, gout, lam);
  return hipGetLastError();
}

hipError_t launch_readout_face(int64_t C, const FaceMap &f, const float *S, const int32_t *dirs, int nout,
                               float *out, hipStream_t s) {
  const int64_t total = (int64_t)f.count * nout * 4;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(readout_face_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, C, f, S, dirs, nout, out);
  return hipGetLastError();
}

hipError_t launch_readout_face_adjoint(int64_t C, const FaceMap &f, const int32_t *dirs, int nout,
                                       const float *gout, float *lam, hipStream_t s) {
  const int64_t total = (int64_t)f.count * nout * 4;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(readout_face_adjoint_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, C, f, dirs, nout,
                     gout, lam);
  return hipGetLastError();
}

int sums_partials(const Geometry &g) { return (int)grid_for(g.C, kSumThreads, 1024); }

// ---- allocation-free totals ---------------------------------------------------
// The float64 partial sums of rt_totals_noalloc live in a static device array
// instead of the caller's workspace: 4 sums per block of sums_kernel, at most
// kScratchPartials blocks (sums_partials never asks for more).  Each device
// holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device, kept per device below.
constexpr int kScratchPartials = 1024;
static __device__ __align__(256) double scratch[4 * kScratchPartials];

namespace {
constexpr int kMaxDevices = 64;
std::atomic<double *> g_scratch[kMaxDevices];
}  // namespace

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch[device].load(std::memory_order_acquire) != nullptr) return hipSuccess;
  double *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr) return hipErrorInvalidSymbol;
  g_scratch[device].store(ptr, std::memory_order_release);
  return hipSuccess;
}

int scratch_partials_max() { return kScratchPartials; }

hipError_t launch_sums_noalloc(const Geometry &g, int device, const float *S, double *result, hipStream_t s) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  double *partial = g_scratch[device].load(std::memory_order_acquire);
  if (partial == nullptr) return hipErrorNotInitialized;
  const int npart = sums_partials(g);
  if (npart > kScratchPartials) return hipErrorInvalidValue;
  // every partial this launch reads is written by it first: nothing to clear
  hipLaunchKernelGGL(sums_kernel, dim3(npart), dim3(kSumThreads), 0, s, g, S, partial);
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(64), 0, s, partial, npart, result);
  return hipGetLastError();
}

hipError_t launch_sums(const Geometry &g, const float *S, double *partial, int npart, double *result,
                       hipStream_t s) {
  hipLaunchKernelGGL(sums_kernel, dim3(npart), dim3(kSumThreads), 0, s, g, S, partial);
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(64), 0, s, partial, npart, result);
  return hipGetLastError();
}

hipError_t launch_maps(const Geometry &g, const float *S, float *I_mean, float *dop_mean, hipStream_t s) {
  hipLaunchKernelGGL(maps_kernel, dim3(grid_for(g.C, 256)), dim3(256), 0, s, g, S, I_mean, dop_mean);
  return hipGetLastError();
}

}  // namespace rtl
