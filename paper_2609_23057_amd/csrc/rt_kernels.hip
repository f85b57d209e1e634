// Device kernels of the polarized lattice-Boltzmann radiative-transfer solver, gfx950.
//
// State layout: planes p = 4 d + s (direction d, Stokes s), each a row-major
// ny x nx float32 array; plane p starts at p * C, C = nx * ny.
//
// The hot kernel is `fused_kernel`: one time step for a tile of 32*CB
// consecutive cells and all 4n rows (direction x Stokes) of those cells.
//  1. Every wave owns one 32-row tile of the contraction and gathers, for its
//     rows and the tile's cells, the streamed state (bilinear pull of Eq. 34
//     from the previous post-collision field, with periodic / absorbing /
//     inflow edges) plus the emission (Eq. 6/8).  The lane mapping of this
//     load is the accumulator layout of a 32x32 MFMA tile, so the values stay
//     in registers for the epilogue.
//  2. The waves write their rows into one LDS tile B[cell][row] in the
//     contraction precision; after a barrier every wave multiplies its 32
//     rows of the collision matrix (read as pre-swizzled lane fragments from
//     L2-resident global memory, only the K range that holds non-zeros) by
//     the whole B tile on the matrix cores (Eq. 25/30).
//  3. Epilogue in float32: Y = alpha X + beta (M X) (absorption and survival,
//     Sec. 2.1.4-2.1.5, Eq. 11), stored as the next post-collision field.
// Contraction rows are ordered r = s * n + d, so the Rayleigh structure (no
// coupling between I,Q,U and V) leaves whole tiles of zeros that are skipped.
//
// The adjoint kernel is the same skeleton run backwards: the B tile holds the
// reverse-pulled adjoint field mu = L^T lambda, the matrix-core product uses
// M^T, and the epilogue forms lambda = alpha mu + beta M^T mu together with
// the per-cell gradient contributions.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_kernels.h"

namespace rtl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kEdgeXm = 0, kEdgeXp = 1, kEdgeYm = 2, kEdgeYp = 3;

__device__ __forceinline__ int wrap_axis(int v, int n, int per) {
  if (per) {
    if (v < 0) v += n;
    if (v < 0) v += n;
    if (v >= n) v -= n;
  }
  return v;
}

// Forward pull of Eq. 34: sum over taps of w * Y(x - ox, y - oy); a source
// outside the lattice on a non-periodic axis reads the ghost radiance of the
// edge it lies beyond (y edges first), which is zero for absorbing edges.
__device__ __forceinline__ float pull_forward(const float *__restrict__ plane, const Geometry &g,
                                              const DirTaps &tp, int x, int y,
                                              const float *__restrict__ ghost, int r) {
  float v = 0.0f;
#pragma unroll
  for (int bx = 0; bx < 2; ++bx) {
    const float wx = bx ? tp.wx1 : tp.wx0;
    if (wx == 0.0f) continue;
    const int xs = wrap_axis(x - tp.ox0 - bx, g.nx, g.per_x);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const float wy = by ? tp.wy1 : tp.wy0;
      if (wy == 0.0f) continue;
      const int ys = wrap_axis(y - tp.oy0 - by, g.ny, g.per_y);
      float f;
      if (ys < 0) f = ghost[kEdgeYm * g.Rpad + r];
      else if (ys >= g.ny) f = ghost[kEdgeYp * g.Rpad + r];
      else if (xs < 0) f = ghost[kEdgeXm * g.Rpad + r];
      else if (xs >= g.nx) f = ghost[kEdgeXp * g.Rpad + r];
      else f = plane[(int64_t)ys * g.nx + xs];
      v += (wx * wy) * f;
    }
  }
  return v;
}

// Transpose of the linear part of pull_forward: the target cell (x, y) reads
// lambda at (x + ox, y + oy) with the same weights; targets that fall outside
// a non-periodic lattice contribute nothing.
__device__ __forceinline__ float pull_adjoint(const float *__restrict__ plane, const Geometry &g,
                                              const DirTaps &tp, int x, int y) {
  float v = 0.0f;
#pragma unroll
  for (int bx = 0; bx < 2; ++bx) {
    const float wx = bx ? tp.wx1 : tp.wx0;
    if (wx == 0.0f) continue;
    const int xs = wrap_axis(x + tp.ox0 + bx, g.nx, g.per_x);
    if (xs < 0 || xs >= g.nx) continue;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const float wy = by ? tp.wy1 : tp.wy0;
      if (wy == 0.0f) continue;
      const int ys = wrap_axis(y + tp.oy0 + by, g.ny, g.per_y);
      if (ys < 0 || ys >= g.ny) continue;
      v += (wx * wy) * plane[(int64_t)ys * g.nx + xs];
    }
  }
  return v;
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
  int rows_off, taps_off, jrow_off, b_off, red_off, total;
  int strideB;   // bytes per cell row of the B tile
  int tileB;     // bytes of one B tile
};

__host__ __device__ inline LdsLayout lds_layout(int n, int Rpad, int esize, int ntile, int cb, int W,
                                               bool adjoint, bool f16) {
  LdsLayout L;
  int off = 0;
  L.rows_off = off;
  off += Rpad * 4;
  L.taps_off = off;
  off += n * (int)sizeof(DirTaps);
  L.jrow_off = off;
  off += Rpad * 4;
  off = (off + 15) & ~15;
  L.b_off = off;
  L.strideB = Rpad * esize + 16;
  L.tileB = 32 * cb * L.strideB;
  off += ntile * L.tileB;
  L.red_off = off;
  int nred = adjoint ? 3 : (f16 ? 1 : 0);
  off += nred * W * 32 * cb * 4;
  L.total = off;
  return L;
}

__device__ __forceinline__ f32x16 mfma_step_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int PREC, bool GATHER, int CB, bool ADJ, int MAXW>
__global__ void __launch_bounds__(64 * MAXW) fused_kernel(StepArgs a, int64_t ntiles) {
  using T = PrecTraits<PREC>;
  extern __shared__ __align__(16) char smem[];
  const Geometry g = a.geo;
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int col = lane & 31;
  const int h = lane >> 5;
  const LdsLayout L = lds_layout(g.n, g.Rpad, T::esize, T::ntile, CB, W, ADJ, PREC == P_F16);
  RowInfo *s_rows = reinterpret_cast<RowInfo *>(smem + L.rows_off);
  DirTaps *s_taps = reinterpret_cast<DirTaps *>(smem + L.taps_off);
  float *s_jrow = reinterpret_cast<float *>(smem + L.jrow_off);
  char *s_b = smem + L.b_off;
  float *s_red = reinterpret_cast<float *>(smem + L.red_off);

  for (int i = threadIdx.x; i < g.Rpad; i += blockDim.x) {
    s_rows[i] = a.rows[i];
    s_jrow[i] = a.jrow[i];
  }
  for (int i = threadIdx.x; i < g.n; i += blockDim.x) s_taps[i] = a.taps[i];
  __syncthreads();

  const int t = w;  // the 32-row tile this wave owns
  const TileRange tr = a.tiles[t];
  constexpr int NC = 32 * CB;

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
    const int64_t c0 = tile * NC;
    float xv[CB][16];
    float mv[ADJ ? CB : 1][16];
    float cscale[CB];
    (void)mv;

    // ---- 1. gather own rows ------------------------------------------------
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int64_t c = c0 + cb * 32 + col;
      const bool valid = c < g.C;
      const int y = valid ? (int)(c / g.nx) : 0;
      const int x = valid ? (int)(c - (int64_t)y * g.nx) : 0;
      const float em = valid ? a.emis[c] : 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = t * 32 + acc_row(i, h);
        const RowInfo ri = s_rows[r];
        float xval = 0.0f, mval = 0.0f;
        if (valid && ri.plane >= 0) {
          const DirTaps tp = s_taps[ri.dir];
          const float *pl = a.in + (int64_t)ri.plane * g.C;
          float sv;
          if (GATHER) sv = pull_forward(pl, g, tp, x, y, a.ghost, r);
          else sv = pl[c];
          if (!ADJ && a.s_out) a.s_out[(int64_t)ri.plane * g.C + c] = sv;
          xval = sv + a.dt_pre * em * s_jrow[r];
          if (ADJ) mval = pull_adjoint(a.lam_next + (int64_t)ri.plane * g.C, g, tp, x, y);
        }
        xv[cb][i] = xval;
        if (ADJ) mv[cb][i] = mval;
      }
    }

    // ---- 1b. per-cell power-of-two scale for fp16 operands -------------------
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) cscale[cb] = 1.0f;
    if (PREC == P_F16) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        float m = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) m = fmaxf(m, fabsf(ADJ ? mv[cb][i] : xv[cb][i]));
        m = fmaxf(m, __shfl_xor(m, 32));
        if (h == 0) s_red[w * NC + cb * 32 + col] = m;
      }
      __syncthreads();
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        float m = 0.0f;
        for (int ww = 0; ww < W; ++ww) m = fmaxf(m, s_red[ww * NC + cb * 32 + col]);
        int e = 0;
        if (m > 0.0f) (void)frexpf(m, &e);
        cscale[cb] = (m > 0.0f) ? ldexpf(1.0f, 8 - e) : 1.0f;
      }
    }

    // ---- 2. rows -> LDS B tile -------------------------------------------------
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      char *brow = s_b + (cb * 32 + col) * L.strideB;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r0 = t * 32 + q * 8 + h * 4;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = ADJ ? mv[cb][4 * q + j] : xv[cb][4 * q + j];
        if (PREC == P_F32) {
          *reinterpret_cast<f32x4 *>(brow + r0 * 4) = f32x4{v[0], v[1], v[2], v[3]};
        } else if (PREC == P_BF16 || PREC == P_BF16X3) {
          bf16x4 hi;
#pragma unroll
          for (int j = 0; j < 4; ++j) hi[j] = static_cast<__bf16>(v[j]);
          *reinterpret_cast<bf16x4 *>(brow + r0 * 2) = hi;
          if (PREC == P_BF16X3) {
            bf16x4 lo;
#pragma unroll
            for (int j = 0; j < 4; ++j) lo[j] = static_cast<__bf16>(v[j] - static_cast<float>(hi[j]));
            *reinterpret_cast<bf16x4 *>(brow + L.tileB + r0 * 2) = lo;
          }
        } else {
          f16x4 hv;
#pragma unroll
          for (int j = 0; j < 4; ++j) hv[j] = static_cast<_Float16>(v[j] * cscale[cb]);
          *reinterpret_cast<f16x4 *>(brow + r0 * 2) = hv;
        }
      }
    }
    __syncthreads();

    // ---- 3. matrix-core contraction over the tile's K range ------------------
    f32x16 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = f32x16{0};
    if (PREC == P_F32) {
      int rec = tr.frag_off;
      for (int kb = tr.klo; kb < tr.khi; kb += 8, rec += 64) {
        const f32x4 av = *reinterpret_cast<const f32x4 *>(a.frag + rec + lane);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const f32x4 bv = *reinterpret_cast<const f32x4 *>(s_b + (cb * 32 + col) * L.strideB +
                                                            (kb + 4 * h) * 4);
          acc[cb] = mfma_step_f32(av[0], bv[0], acc[cb]);
          acc[cb] = mfma_step_f32(av[1], bv[1], acc[cb]);
          acc[cb] = mfma_step_f32(av[2], bv[2], acc[cb]);
          acc[cb] = mfma_step_f32(av[3], bv[3], acc[cb]);
        }
      }
    } else {
      int rec = tr.frag_off;
      for (int kb = tr.klo; kb < tr.khi; kb += 16, rec += 64) {
        const uint4 araw = a.frag[rec + lane];
        uint4 araw_lo;
        if (PREC == P_BF16X3) araw_lo = a.frag_lo[rec + lane];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const char *bp = s_b + (cb * 32 + col) * L.strideB + (kb + 8 * h) * 2;
          if (PREC == P_F16) {
            const f16x8 av = __builtin_bit_cast(f16x8, araw);
            const f16x8 bv = *reinterpret_cast<const f16x8 *>(bp);
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc[cb], 0, 0, 0);
          } else {
            const bf16x8 av = __builtin_bit_cast(bf16x8, araw);
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(bp);
            if (PREC == P_BF16X3) {
              const bf16x8 alo = __builtin_bit_cast(bf16x8, araw_lo);
              const bf16x8 blo = *reinterpret_cast<const bf16x8 *>(bp + L.tileB);
              acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bv, acc[cb], 0, 0, 0);
              acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, blo, acc[cb], 0, 0, 0);
            }
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[cb], 0, 0, 0);
          }
        }
      }
    }

    // ---- 4. epilogue -------------------------------------------------------------
    float part[3][CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      part[0][cb] = part[1][cb] = part[2][cb] = 0.0f;
      const int64_t c = c0 + cb * 32 + col;
      if (c < g.C) {
        const float al = a.alpha[c], be = a.beta[c];
        const float em = a.emis[c];
        const float unscale = a.a_scale_inv / cscale[cb];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int r = t * 32 + acc_row(i, h);
          const RowInfo ri = s_rows[r];
          if (ri.plane < 0) continue;
          const float prod = acc[cb][i] * unscale;
          if (!ADJ) {
            const float yv = al * xv[cb][i] + be * prod + a.dt_post * em * s_jrow[r];
            a.out[(int64_t)ri.plane * g.C + c] = yv;
          } else {
            const float lam = al * mv[cb][i] + be * prod;
            a.out[(int64_t)ri.plane * g.C + c] = lam;
            part[0][cb] += mv[cb][i] * xv[cb][i];
            part[1][cb] += prod * xv[cb][i];
            part[2][cb] += (a.dt_pre * lam + a.dt_post * mv[cb][i]) * s_jrow[r];
          }
        }
      }
    }
    if (ADJ) {
      // per-cell sums over all rows: half-waves, then waves via LDS
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          float v = part[k][cb];
          v += __shfl_xor(v, 32);
          if (h == 0) s_red[(k * W + w) * NC + cb * 32 + col] = v;
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 3 * NC; e += blockDim.x) {
        const int k = e / NC, cc = e - k * NC;
        const int64_t c = c0 + cc;
        if (c < g.C) {
          double s = 0.0;
          for (int ww = 0; ww < W; ++ww) s += (double)s_red[(k * W + ww) * NC + cc];
          a.gacc[(int64_t)k * g.C + c] += s;
        }
      }
    }
    __syncthreads();
  }
}

template <int PREC, bool GATHER, int CB, bool ADJ>
hipError_t launch_fused_t(const StepArgs &a, int W, hipStream_t s, int grid_limit) {
  using T = PrecTraits<PREC>;
  const LdsLayout L = lds_layout(a.geo.n, a.geo.Rpad, T::esize, T::ntile, CB, W, ADJ, PREC == P_F16);
  const int64_t ntiles = (a.geo.C + 32 * CB - 1) / (32 * CB);
  int64_t grid = ntiles;
  if (grid > grid_limit) grid = grid_limit;
  if (grid >= 8) grid &= ~7LL;
  if (grid < 1) grid = 1;
  if (W <= 4) {
    auto k = fused_kernel<PREC, GATHER, CB, ADJ, 4>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * W), L.total, s, a, ntiles);
  } else {
    auto k = fused_kernel<PREC, GATHER, CB, ADJ, 16>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * W), L.total, s, a, ntiles);
  }
  return hipGetLastError();
}

template <bool ADJ>
hipError_t launch_fused(const StepArgs &a, int prec, bool gather, int cb, hipStream_t s, int grid_limit) {
  const int W = a.geo.Rpad / 32;
  if (W < 1 || W > 16) return hipErrorInvalidValue;
#define RT_DISPATCH(P)                                                                       \
  if (prec == P) {                                                                           \
    if (gather) return cb == 2 ? launch_fused_t<P, true, 2, ADJ>(a, W, s, grid_limit)        \
                               : launch_fused_t<P, true, 1, ADJ>(a, W, s, grid_limit);       \
    return cb == 2 ? launch_fused_t<P, false, 2, ADJ>(a, W, s, grid_limit)                   \
                   : launch_fused_t<P, false, 1, ADJ>(a, W, s, grid_limit);                  \
  }
  RT_DISPATCH(P_F32)
  RT_DISPATCH(P_BF16)
  RT_DISPATCH(P_F16)
  RT_DISPATCH(P_BF16X3)
#undef RT_DISPATCH
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- plain path --

// S_out[p](x, y) = pull_forward(S_in[p]) for every plane p = blockIdx.y.
__global__ void __launch_bounds__(256) stream_kernel(StepArgs a, const float *__restrict__ in,
                                                     float *__restrict__ out) {
  const Geometry g = a.geo;
  const int p = blockIdx.y;
  const int d = p >> 2, s = p & 3;
  const int r = s * g.n + d;
  const DirTaps tp = a.taps[d];
  const float *pl = in + (int64_t)p * g.C;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(c / g.nx);
    const int x = (int)(c - (int64_t)y * g.nx);
    out[(int64_t)p * g.C + c] = pull_forward(pl, g, tp, x, y, a.ghost, r);
  }
}

// Y(c) = alpha X(c) + beta M X(c) + dt_post J(c), X = S + dt_pre J, one
// thread per cell, M in ABI order (row 4 d_out + s_out) read with uniform
// (scalar) loads.
__global__ void __launch_bounds__(256) collide_valu_kernel(StepArgs a, const float *__restrict__ M,
                                                           const float *__restrict__ in,
                                                           float *__restrict__ out) {
  const Geometry g = a.geo;
  const int n = g.n, R = g.R;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const float al = a.alpha[c], be = a.beta[c], em = a.emis[c];
    for (int dout = 0; dout < n; ++dout) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      for (int di = 0; di < n; ++di) {
        float xs[4];
#pragma unroll
        for (int si = 0; si < 4; ++si)
          xs[si] = in[(int64_t)(4 * di + si) * g.C + c] + a.dt_pre * em * a.jrow[si * n + di];
        const float *mrow = M + (int64_t)(4 * dout) * R + 4 * di;
#pragma unroll
        for (int so = 0; so < 4; ++so)
#pragma unroll
          for (int si = 0; si < 4; ++si) acc[so] += mrow[so * R + si] * xs[si];
      }
#pragma unroll
      for (int so = 0; so < 4; ++so) {
        const int64_t off = (int64_t)(4 * dout + so) * g.C + c;
        const float jr = a.jrow[so * n + dout];
        const float xo = in[off] + a.dt_pre * em * jr;
        out[off] = al * xo + be * acc[so] + a.dt_post * em * jr;
      }
    }
  }
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

__global__ void gradchain_kernel(int64_t C, const float *__restrict__ tau, const float *__restrict__ alb,
                                 uint32_t flags, const double *__restrict__ gacc, float *g_tau,
                                 float *g_alb, float *g_emis) {
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
    if (g_tau) g_tau[c] = (float)(ga * dat + gb * dbt);
    if (g_alb) g_alb[c] = (float)(ga * daw + gb * dbw);
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

size_t step_lds_bytes(const Geometry &g, int prec, int cb, bool adjoint) {
  const int esize = prec == P_F32 ? 4 : 2;
  const int ntile = prec == P_BF16X3 ? 2 : 1;
  const LdsLayout L = lds_layout(g.n, g.Rpad, esize, ntile, cb, g.Rpad / 32, adjoint, prec == P_F16);
  return (size_t)L.total;
}

hipError_t launch_step_mfma(const StepArgs &a, int prec, bool gather, int cb, hipStream_t s,
                            int grid_limit) {
  return launch_fused<false>(a, prec, gather, cb, s, grid_limit);
}

hipError_t launch_adjoint_mfma(const StepArgs &a, int prec, bool gather, int cb, hipStream_t s,
                               int grid_limit) {
  return launch_fused<true>(a, prec, gather, cb, s, grid_limit);
}

hipError_t launch_stream(const StepArgs &a, const float *in, float *out, hipStream_t s) {
  dim3 grid(grid_for(a.geo.C, 256, 1024), 4 * a.geo.n);
  hipLaunchKernelGGL(stream_kernel, grid, dim3(256), 0, s, a, in, out);
  return hipGetLastError();
}

hipError_t launch_collide_valu(const StepArgs &a, const float *M_abi, const float *in, float *out,
                               hipStream_t s) {
  hipLaunchKernelGGL(collide_valu_kernel, dim3(grid_for(a.geo.C, 256)), dim3(256), 0, s, a, M_abi, in,
                     out);
  return hipGetLastError();
}

hipError_t launch_coef(int64_t C, const float *tau, const float *alb, const float *emis, float *tau_c,
                       float *alb_c, float *emis_c, float *alpha, float *beta, uint32_t flags, int *bad,
                       hipStream_t s) {
  hipLaunchKernelGGL(coef_kernel, dim3(grid_for(C, 256)), dim3(256), 0, s, C, tau, alb, emis, tau_c,
                     alb_c, emis_c, alpha, beta, flags, bad);
  return hipGetLastError();
}

hipError_t launch_gradchain(int64_t C, const float *tau, const float *alb, uint32_t flags,
                            const double *gacc, float *g_tau, float *g_alb, float *g_emis,
                            hipStream_t s) {
  hipLaunchKernelGGL(gradchain_kernel, dim3(grid_for(C, 256)), dim3(256), 0, s, C, tau, alb, flags,
                     gacc, g_tau, g_alb, g_emis);
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

int sums_partials(const Geometry &g) { return (int)grid_for(g.C, kSumThreads, 1024); }

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
