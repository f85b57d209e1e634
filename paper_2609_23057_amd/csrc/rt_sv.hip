// Statevector emulation kernels (gfx950): the gates of the paper's circuit on
// a real float64 statevector.  A gate alone, or a run of gates on at most 3
// target qubits, is one pass over the states it touches, so each kernel is
// bound by HBM traffic (16 bytes read and 16 written per amplitude pair of a
// gate alone, per amplitude of a fused run); threads walk their index space
// with a grid-stride loop, consecutive threads on consecutive states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rt_sv.h"

namespace rtl {

namespace {

constexpr int kSvThreads = 256;
constexpr int kSvNormBlocks = 1024;

inline unsigned sv_grid(uint64_t work) {
  const uint64_t b = (work + kSvThreads - 1) / kSvThreads;
  return (unsigned)std::min<uint64_t>(std::max<uint64_t>(b, 1), 65536);
}

// Index with zero bits inserted at the (ascending) fixed positions of the
// gate (its pair and control qubits), then the control values set.
__device__ __forceinline__ uint64_t insert_fixed(uint64_t t, const SvGate &g) {
  for (int k = 0; k < g.nfixed; ++k) {
    const int p = g.fixed[k];
    t = ((t >> p) << (p + 1)) | (t & ((1ull << p) - 1));
  }
  return t | g.cval;
}

__global__ void __launch_bounds__(kSvThreads) sv_gate_kernel(double *__restrict__ psi, uint64_t npairs, SvGate g) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npairs; t += stride) {
    const uint64_t base = insert_fixed(t, g);
    uint32_t a = 0;
    for (int j = 0; j < g.naddr; ++j) a |= (uint32_t)((base >> g.addr[j]) & 1) << j;
    const double u00 = g.table[4 * a], u01 = g.table[4 * a + 1];
    const double u10 = g.table[4 * a + 2], u11 = g.table[4 * a + 3];
    const uint64_t i = base | g.v0, k = base | g.v1;
    const double a0 = (g.v0 & g.zread) ? 0.0 : psi[i];
    const double a1 = (g.v1 & g.zread) ? 0.0 : psi[k];
    // products then sums, unfused, as the reference arithmetic does
    psi[i] = u00 * a0 + u01 * a1;
    psi[k] = u10 * a0 + u11 * a1;
  }
}

// One pair (i0, i1) of the local amplitudes under gate fg (full index of
// the local state j: base | spread(j)); compile-time local indices keep amp
// in registers.
template <int M>
__device__ __forceinline__ uint64_t sv_spread(int j, const SvFuse &f) {
  uint64_t v = 0;
#pragma unroll
  for (int k = 0; k < M; ++k) v |= (uint64_t)((j >> k) & 1) << f.tq[k];
  return v;
}

template <int M, int LV0, int LV1, int LMASK>
__device__ __forceinline__ void sv_apply_local(double (&amp)[1 << M], uint64_t base, const SvFusedGate &fg,
                                               const SvFuse &f) {
#pragma unroll
  for (int j = 0; j < (1 << M); ++j) {
    if ((j & LMASK) != 0) continue;
    const uint64_t full = base | sv_spread<M>(j, f);
    if ((full & fg.cmask) != fg.cval) continue;
    uint32_t a = 0;
    for (int q = 0; q < fg.naddr; ++q) a |= (uint32_t)((full >> fg.addr[q]) & 1) << q;
    const double u00 = fg.table[4 * a], u01 = fg.table[4 * a + 1];
    const double u10 = fg.table[4 * a + 2], u11 = fg.table[4 * a + 3];
    const double a0 = amp[j | LV0], a1 = amp[j | LV1];
    amp[j | LV0] = u00 * a0 + u01 * a1;
    amp[j | LV1] = u10 * a0 + u11 * a1;
  }
}

template <int M>
__global__ void __launch_bounds__(kSvThreads) sv_fused_kernel(double *__restrict__ psi, uint64_t nbases, SvFuse f) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nbases; t += stride) {
    uint64_t base = t;
    for (int k = 0; k < f.nfixed; ++k) {
      const int p = f.fixed[k];
      base = ((base >> p) << (p + 1)) | (base & ((1ull << p) - 1));
    }
    base |= f.ccval;
    double amp[1 << M];
#pragma unroll
    for (int j = 0; j < (1 << M); ++j) amp[j] = (j & f.zlocal) ? 0.0 : psi[base | sv_spread<M>(j, f)];
    for (int gi = 0; gi < f.ngates; ++gi) {
      const SvFusedGate &fg = f.g[gi];
      switch (fg.code) {
        case 0: sv_apply_local<M, 0, 1, 1>(amp, base, fg, f); break;
        case 1: if constexpr (M > 1) sv_apply_local<M, 0, 2, 2>(amp, base, fg, f); break;
        case 2: if constexpr (M > 2) sv_apply_local<M, 0, 4, 4>(amp, base, fg, f); break;
        case 3 + 3 * 0 + 1: if constexpr (M > 1) sv_apply_local<M, 1, 2, 3>(amp, base, fg, f); break;
        case 3 + 3 * 1 + 0: if constexpr (M > 1) sv_apply_local<M, 2, 1, 3>(amp, base, fg, f); break;
        case 3 + 3 * 0 + 2: if constexpr (M > 2) sv_apply_local<M, 1, 4, 5>(amp, base, fg, f); break;
        case 3 + 3 * 2 + 0: if constexpr (M > 2) sv_apply_local<M, 4, 1, 5>(amp, base, fg, f); break;
        case 3 + 3 * 1 + 2: if constexpr (M > 2) sv_apply_local<M, 2, 4, 6>(amp, base, fg, f); break;
        case 3 + 3 * 2 + 1: if constexpr (M > 2) sv_apply_local<M, 4, 2, 6>(amp, base, fg, f); break;
        default: break;
      }
    }
#pragma unroll
    for (int j = 0; j < (1 << M); ++j) psi[base | sv_spread<M>(j, f)] = amp[j];
  }
}

__global__ void __launch_bounds__(kSvThreads) sv_shift_kernel(const double *__restrict__ in, double *__restrict__ out,
                                                             uint64_t nstates, SvShift s) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const int64_t size = 1ll << s.qr;
  const uint64_t rmask = (uint64_t)(size - 1) << s.r0;
  for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < nstates; o += stride) {
    if ((o & s.zmask) != 0) {   // its source has the same zero qubit
      out[o] = 0.0;
      continue;
    }
    uint64_t src = o;
    if (((o >> s.slbit) & 1) == 0) {
      const int64_t r = (int64_t)((o >> s.r0) & (uint64_t)(size - 1));
      const int e = (int)((o >> s.ebit) & 1);
      const int k = (int)((o >> s.d0) & ((1u << s.qd) - 1));
      const int64_t t = (int64_t)s.base[k] + (int64_t)((o >> s.abit) & 1);
      const int64_t back = (r - t) & (size - 1);   // (r - t) mod size (size a power of two)
      int64_t rs = r;
      int es = e;
      if (s.periodic) {
        rs = back;
      } else if (e == 0) {
        // an unmarked output came from back unless back + t lies outside
        rs = back;
        es = (back + t < 0 || back + t >= size) ? 1 : 0;
      } else {
        // a marked output: the state that stayed in place (marked now)
        es = 1 ^ ((r + t < 0 || r + t >= size) ? 1 : 0);
      }
      src = (o & ~rmask & ~(1ull << s.ebit)) | ((uint64_t)rs << s.r0) | ((uint64_t)es << s.ebit);
    }
    out[o] = (s.ezero && ((src >> s.ebit) & 1)) ? 0.0 : in[src];
  }
}

__global__ void sv_zero_kernel(double *__restrict__ p, uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

__global__ void __launch_bounds__(kSvThreads) sv_norm_partial_kernel(const double *__restrict__ a, uint64_t na,
                                                                     const double *__restrict__ b, uint64_t nb,
                                                                     double *__restrict__ partial) {
  __shared__ double red[kSvThreads];
  double acc = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
    const double v = i < na ? a[i] : b[i - na];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kSvThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block of kSvThreads threads: each sums a strided share of the partials,
// then a tree in LDS (a fixed order, so the result does not vary run to run).
__global__ void __launch_bounds__(kSvThreads) sv_norm_final_kernel(const double *__restrict__ partial, int np,
                                                                   double *result) {
  __shared__ double red[kSvThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kSvThreads) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSvThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = red[0];
}

__device__ __forceinline__ uint64_t data_index(int st, int sl, int din, int dout, int y, int x, int nd, int ny,
                                               int nx) {
  return (((((uint64_t)(st * 2 + sl) * nd + din) * nd + dout) * ny + y) * nx + x);
}

__global__ void sv_encode_kernel(double *__restrict__ psi, const double *__restrict__ S,
                                 const double *__restrict__ J, int n, int nd, int ny, int nx,
                                 const double *__restrict__ norm2) {
  const uint64_t total = (uint64_t)n * 4 * ny * nx;
  const double norm = sqrt(*norm2);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int st = (int)((i / ((uint64_t)nx * ny)) % 4);
    const int d = (int)(i / ((uint64_t)nx * ny * 4));
    psi[data_index(st, 0, d, d, y, x, nd, ny, nx)] = norm > 0.0 ? S[i] / norm : 0.0;
    psi[data_index(st, 1, d, d, y, x, nd, ny, nx)] = norm > 0.0 ? J[i] / norm : 0.0;
  }
}

// Every state of the data block (index < 2^ndata: all ancillas 0):
// (st, sl, d_in, d_out, y, x) from the index, the encoded value where
// d_in = d_out < n, else zero.
__global__ void sv_encode_block_kernel(double *__restrict__ psi, const double *__restrict__ S,
                                       const double *__restrict__ J, int n, int nd, int ny, int nx,
                                       const double *__restrict__ norm2) {
  const uint64_t total = (uint64_t)8 * nd * nd * ny * nx;
  const double norm = sqrt(*norm2);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    uint64_t r = i;
    const int x = (int)(r % nx);
    r /= nx;
    const int y = (int)(r % ny);
    r /= ny;
    const int dout = (int)(r % nd);
    r /= nd;
    const int din = (int)(r % nd);
    r /= nd;
    const int sl = (int)(r % 2);
    const int st = (int)(r / 2);
    double v = 0.0;
    if (din == dout && din < n && norm > 0.0) {
      const uint64_t f = (((uint64_t)din * 4 + st) * ny + y) * nx + x;
      v = (sl == 0 ? S[f] : J[f]) / norm;
    }
    psi[i] = v;
  }
}

__global__ void sv_decode_kernel(const double *__restrict__ psi, double *__restrict__ S, int n, int nd, int ny,
                                 int nx, double scale2, const double *__restrict__ norm2) {
  const uint64_t total = (uint64_t)n * 4 * ny * nx;
  const double scale = scale2 * sqrt(*norm2);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int st = (int)((i / ((uint64_t)nx * ny)) % 4);
    const int k = (int)(i / ((uint64_t)nx * ny * 4));
    double acc = 0.0;
    for (int din = 0; din < nd; ++din) acc += psi[data_index(st, 0, din, k, y, x, nd, ny, nx)];
    S[i] = acc * scale;
  }
}

}  // namespace

hipError_t sv_launch_gate(double *psi, int nq, const SvGate &gate, hipStream_t s) {
  SvGate g = gate;
  if (g.nbits < 1 || g.nbits > 2 || g.naddr < 0 || g.naddr > kSvMaxAddr || nq > 40) return hipErrorInvalidValue;
  if ((g.mask & g.cmask) != 0 || (g.cval & ~g.cmask) != 0 || (g.mask | g.cmask) >> nq != 0) return hipErrorInvalidValue;
  g.nfixed = 0;
  for (int b = 0; b < nq; ++b)
    if (((g.mask | g.cmask) >> b) & 1) {
      if (g.nfixed == 24) return hipErrorInvalidValue;
      g.fixed[g.nfixed++] = b;
    }
  const uint64_t npairs = 1ull << (nq - g.nfixed);
  hipLaunchKernelGGL(sv_gate_kernel, dim3(sv_grid(npairs)), dim3(kSvThreads), 0, s, psi, npairs, g);
  return hipGetLastError();
}

hipError_t sv_launch_fused(double *psi, int nq, const SvFuse &fuse, hipStream_t s) {
  SvFuse f = fuse;
  if (f.m < 1 || f.m > kSvFuseMaxQ || f.ngates < 1 || f.ngates > kSvFuseMaxGates || nq > 40 || nq < f.m)
    return hipErrorInvalidValue;
  uint64_t tmask = 0;
  for (int k = 0; k < f.m; ++k) {
    if (f.tq[k] < 0 || f.tq[k] >= nq || (k > 0 && f.tq[k] <= f.tq[k - 1])) return hipErrorInvalidValue;
    tmask |= 1ull << f.tq[k];
  }
  if ((f.ccmask & tmask) != 0 || (f.ccval & ~f.ccmask) != 0 || (f.ccmask >> nq) != 0) return hipErrorInvalidValue;
  f.nfixed = 0;
  for (int b = 0; b < nq; ++b)
    if (((tmask | f.ccmask) >> b) & 1) {
      if (f.nfixed == kSvFuseMaxQ + 16) return hipErrorInvalidValue;
      f.fixed[f.nfixed++] = b;
    }
  for (int i = 0; i < f.ngates; ++i) {
    const SvFusedGate &g = f.g[i];
    const int c = g.code;
    const bool one = c >= 0 && c < f.m;
    const bool two = c >= 3 && c < 12 && (c - 3) / 3 != (c - 3) % 3 && (c - 3) / 3 < f.m && (c - 3) % 3 < f.m;
    if (!(one || two) || g.naddr < 0 || g.naddr > kSvMaxAddr || (g.cval & ~g.cmask) != 0 || g.cmask >> nq != 0)
      return hipErrorInvalidValue;
    // a gate's own target qubits are not among its controls
    const int ta = one ? c : (c - 3) / 3, tb = one ? c : (c - 3) % 3;
    if (((g.cmask >> f.tq[ta]) & 1) || ((g.cmask >> f.tq[tb]) & 1)) return hipErrorInvalidValue;
    for (int q = 0; q < g.naddr; ++q)
      if (g.addr[q] < 0 || g.addr[q] >= nq) return hipErrorInvalidValue;
  }
  const uint64_t nbases = 1ull << (nq - f.nfixed);
  const dim3 grid(sv_grid(nbases)), block(kSvThreads);
  if (f.m == 1) hipLaunchKernelGGL(sv_fused_kernel<1>, grid, block, 0, s, psi, nbases, f);
  if (f.m == 2) hipLaunchKernelGGL(sv_fused_kernel<2>, grid, block, 0, s, psi, nbases, f);
  if (f.m == 3) hipLaunchKernelGGL(sv_fused_kernel<3>, grid, block, 0, s, psi, nbases, f);
  return hipGetLastError();
}

hipError_t sv_launch_shift(const double *in, double *out, int nq, const SvShift &t, hipStream_t s) {
  if (nq > 40 || t.qr < 1 || t.qd < 1) return hipErrorInvalidValue;
  // the zero qubits lie outside the translated register and the escape marker
  const uint64_t moved = (((1ull << t.qr) - 1) << t.r0) | (1ull << t.ebit);
  if ((t.zmask & moved) != 0 || (t.zmask >> nq) != 0) return hipErrorInvalidValue;
  const uint64_t n = 1ull << nq;
  hipLaunchKernelGGL(sv_shift_kernel, dim3(sv_grid(n)), dim3(kSvThreads), 0, s, in, out, n, t);
  return hipGetLastError();
}

hipError_t sv_launch_zero(double *psi, uint64_t count, hipStream_t s) {
  hipLaunchKernelGGL(sv_zero_kernel, dim3(sv_grid(count)), dim3(kSvThreads), 0, s, psi, count);
  return hipGetLastError();
}

int sv_norm_partials() { return kSvNormBlocks; }

hipError_t sv_launch_norm2(const double *a, uint64_t na, const double *b, uint64_t nb, double *partial,
                           double *result, hipStream_t s) {
  hipLaunchKernelGGL(sv_norm_partial_kernel, dim3(kSvNormBlocks), dim3(kSvThreads), 0, s, a, na, b, nb, partial);
  hipLaunchKernelGGL(sv_norm_final_kernel, dim3(1), dim3(kSvThreads), 0, s, partial, kSvNormBlocks, result);
  return hipGetLastError();
}

hipError_t sv_launch_encode(double *psi, const double *S, const double *J, int n, int nd, int ny, int nx,
                            const double *norm2, hipStream_t s) {
  const uint64_t total = (uint64_t)n * 4 * ny * nx;
  hipLaunchKernelGGL(sv_encode_kernel, dim3(sv_grid(total)), dim3(kSvThreads), 0, s, psi, S, J, n, nd, ny, nx,
                     norm2);
  return hipGetLastError();
}

hipError_t sv_launch_encode_block(double *psi, const double *S, const double *J, int n, int nd, int ny, int nx,
                                  const double *norm2, hipStream_t s) {
  const uint64_t total = (uint64_t)8 * nd * nd * ny * nx;
  hipLaunchKernelGGL(sv_encode_block_kernel, dim3(sv_grid(total)), dim3(kSvThreads), 0, s, psi, S, J, n, nd, ny, nx,
                     norm2);
  return hipGetLastError();
}

hipError_t sv_launch_decode(const double *psi, double *S, int n, int nd, int ny, int nx, double scale2,
                            const double *norm2, hipStream_t s) {
  const uint64_t total = (uint64_t)n * 4 * ny * nx;
  hipLaunchKernelGGL(sv_decode_kernel, dim3(sv_grid(total)), dim3(kSvThreads), 0, s, psi, S, n, nd, ny, nx,
                     scale2, norm2);
  return hipGetLastError();
}

}  // namespace rtl
