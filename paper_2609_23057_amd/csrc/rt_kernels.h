// Device kernel launchers of the polarized LBM solver (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_internal.h"

namespace rtl {

// Optional extensions of the fused step: a per-cell mixture of phase
// functions (further contractions) or dichroic absorption (in the gather).
enum { kExtNone = 0, kExtMix = 1, kExtDich = 2 };

struct Geometry {
  int64_t C;       // cells nx * ny
  int32_t nx, ny;
  int32_t per_x, per_y;   // periodic axes
  int32_t n, R, Rpad;
};

// Everything a fused forward or adjoint launch needs.
struct StepArgs {
  Geometry geo;
  const DirTaps *taps;     // [n]
  const float *jrow;       // [Rpad] emission profile j[d][s] at row 4 d + s (zero padded)
  const float *ghost;      // [5][Rpad] ghost radiance per edge and row 4 d + s (0 if not inflow),
                           // then a row of zeros
  const float *alpha, *beta, *emis;   // [C]
  float dt_pre;            // dt * e: emission added before the collision
  float dt_post;           // dt * (1 - e): emission added after it (fused Taylor)
  const uint4 *frag;       // A fragments (M for forward, M^T for adjoint)
  const uint4 *frag_lo;    // low bf16 parts of A for BF16 and BF16X3
  const TileRange *tiles;  // [Rpad / 32]
  float a_scale_inv;       // 1 / global scale of A (FP16)
  // forward
  const float *in;         // gather source (Y_{t-1}) or direct state S_t
  float *out;              // Y_t (forward) / lambda_t (adjoint)
  float *s_out;            // optional streamed state S_t (forward)
  // adjoint
  const float *lam_next;   // lambda_{t+1}
  double *gacc;            // [3][C]: g_alpha, g_beta, g_emis accumulators
  // phase mixture (frac == nullptr: none): the scattering of cell c follows
  // the further matrix M_j (j < nmix) with weight frac[j C + c] and M with
  // the rest, 1 - sum_j frac[j C + c]; the adjoint step takes M_j^T here as
  // it takes M^T in frag / tiles.  Component j's fragments start at
  // frag2 + j frag2_stride (its low parts likewise), its tiles at
  // tiles2 + j (Rpad / 32), its plain-path matrix at MT2 + j R R.
  const uint4 *frag2;      // A fragments of the M_j (M_j^T), in the contraction precision
  const uint4 *frag2_lo;   // bf16 and bf16x3: their low parts
  const TileRange *tiles2; // [nmix][Rpad / 32]
  const float *frac;       // [nmix][C]
  const float *MT2;        // plain path: float32 M_j transposed [nmix][R][R] (row k holds M_j[r][k] for all r)
  int32_t nmix;            // further matrices, >= 1 when frac is set
  int64_t frag2_stride;    // uint4 records between components' fragments
  // dichroic absorption (forward only; dich_xi == nullptr: none): I + Q and
  // I - Q of direction d in cell c are multiplied by exp(-+dich_xi[c] dich_w[d])
  const float *dich_xi;    // [C] tau_abs * eta per cell
  const float *dich_w;     // [n] sin^2 theta_d
  // 3-D lattice (geo.ny = ny3 * nz rows of nx cells): the fused forward step
  // with the trilinear pull in its gather (ghost then holds the face table
  // [7][Rpad]); its tiles are 32-cell runs of one row, taken in blocks of
  // zblk layers with the layer index fastest
  int32_t ny3, nz, per_z, zblk;
  const DirTaps3 *taps3;   // [n]
  // 2-D single-problem steps: tiles walk vertical strips (strip tiles of 64
  // cells across, or strip / 2 tiles of 32 cells; every row, then the next
  // strip); 0: row order.  Set only where nx is a multiple of 64 strip.
  int32_t strip;
  // single-problem forward steps without extensions (64-cell tiles, 16-wave
  // blocks, 3-D) write the output state with non-temporal stores: set for
  // states beyond the last-level cache, which the next step cannot find
  // there anyway (below it such stores would push the state out of it)
  int32_t nt_out;
};

enum Prec { P_F32 = 0, P_BF16 = 1, P_F16 = 2, P_BF16X3 = 3 };

// ---- spectral batch ----------------------------------------------------------
// Buffers of a channel by id; a batched launch names, for every role (input,
// output, checkpoint store, adjoint lambda), one id and a slot, the same for
// all channels.  Slotted buffers hold consecutive states of the channel.
enum BatchBuf {
  kBufNone = -1,
  kBufS = 0,     // caller's state
  kBufYa = 1,    // post-collision ping-pong buffers (workspace)
  kBufYb = 2,
  kBufCkpt = 3,  // caller's checkpoints (slotted)
  kBufSeg = 4,   // caller's segment buffer (slotted)
  kBufLamT = 5,  // caller's lambda_T
  kBufLa = 6,    // adjoint ping-pong buffers (workspace)
  kBufLb = 7,
  kBufCount = 8
};

struct BatchChan {
  StepArgs a;            // operators and per-cell tables of the channel (role pointers unused)
  float *buf[kBufCount]; // buffers by id
  int64_t state_elems;   // floats of one state (stride of slotted buffers)
  int64_t item0;         // first work item of the channel
  int64_t ntiles;        // 32-cell tiles
  int32_t groups;        // tile groups per work item (block waves / waves per tile)
  int32_t pad;
};

struct BatchSel {
  int in, out, sout, lam;
  int in_slot, out_slot, sout_slot, lam_slot;
};

// Largest block of the batched kernel, in waves.  A channel needs W = Rpad / 32
// waves per tile; a class of channels with the same W runs in blocks of
// bw waves (bw a multiple of W, at most kBatchWaves): bw / W tiles side by side.
constexpr int kBatchWaves = 8;

// LDS bytes the batched kernel needs for a channel of this padded size in
// blocks of bw waves (SIZE_MAX if bw does not fit the channel).
size_t batch_lds_bytes(int Rpad, int prec, bool adjoint, int bw, bool dich = false);

// Sets the kernel attributes of the bw-wave batched kernels and returns their
// blocks per CU for the given LDS size (called before any stream capture).
hipError_t prepare_batch(int prec, int bw, int lds_bytes, int *blocks_per_cu);

// One batched fused step (forward or adjoint) over the tiles of one class of
// channels in bw-wave blocks; the persistent grid is cu_count x the resident
// blocks of that instantiation.  ext: kExtMix if some channel of the run has
// a phase mixture, kExtDich if some has dichroic absorption (never both; the
// other channels pass through the extension's tile exactly), else kExtNone;
// with kExtDich the adjoint's LDS is batch_lds_bytes(.., dich = true).
hipError_t launch_batch_step(const BatchChan *d_chans, int nchan, int64_t nitems, int prec, int bw, bool adjoint,
                             bool gather, bool ckpt, int ext, const BatchSel &sel, int lds_bytes, int cu_count,
                             hipStream_t s);

// Fused forward step on the matrix cores.  gather: in = Y_{t-1}, X = L(in) +
// dt_pre J; otherwise X = in + dt_pre J.  out = alpha X + beta M X + dt_post J.
// cu_count: compute units of the device (sets the persistent grid).
hipError_t launch_step_mfma(const StepArgs &a, int prec, bool gather, hipStream_t s, int cu_count);

// Fused forward step on a 3-D lattice (float32 contraction): in = Y_{t-1},
// X = L3(in) + dt_pre J with the trilinear pull of the 3-D streaming kernel
// (same taps, same rounding), out = alpha X + beta M X + dt_post J, s_out
// (optional) = L3(in).  hipErrorInvalidValue for another precision, a phase
// mixture or dichroic absorption (those run as collision + streaming).
hipError_t launch_step3_mfma(const StepArgs &a, int prec, hipStream_t s, int cu_count);

// Fused adjoint step: mu = L^T lam_next, X as in the forward, nu = M^T mu,
// out = alpha mu + beta nu, gacc += per-cell (<mu,X>, <nu,X>, dt<.,j>).
hipError_t launch_adjoint_mfma(const StepArgs &a, int prec, bool gather, hipStream_t s,
                               int cu_count);

// Streaming on a 3-D lattice (trilinear pull along x, y and z).
struct Stream3Args {
  int64_t C;                  // nx ny nz
  int32_t nx, ny, nz, n, Rpad;
  int32_t per_x, per_y, per_z;
  const DirTaps3 *taps;       // [n]
  const float *ghost;         // [7][Rpad]: faces x-, x+, y-, y+, z-, z+, then zeros
};
hipError_t launch_stream3d(const Stream3Args &a, const float *in, float *out, hipStream_t s);

// Cells of one face of a 3-D lattice: face cell e = a + na b (a < na) lies at
// base + a sa + b sb; count cells in all.
struct FaceMap {
  int64_t base, sa, sb;
  int32_t na, count;
};
hipError_t launch_readout_face(int64_t C, const FaceMap &f, const float *S, const int32_t *dirs, int nout,
                               float *out, hipStream_t s);
hipError_t launch_readout_face_adjoint(int64_t C, const FaceMap &f, const int32_t *dirs, int nout,
                                       const float *gout, float *lam, hipStream_t s);

// Plain float32 path: separate streaming and vector-ALU collision.
hipError_t launch_stream(const StepArgs &a, const float *in, float *out, hipStream_t s);
hipError_t launch_collide_valu(const StepArgs &a, const float *MT, const float *in, float *out,
                               hipStream_t s);

// Per-cell coefficients from tau/albedo; counts invalid cells into *bad.
hipError_t launch_coef(int64_t C, const float *tau, const float *alb, const float *emis,
                       float *tau_c, float *alb_c, float *emis_c, float *alpha, float *beta,
                       uint32_t flags, int *bad, hipStream_t s);
// Dichroic absorption per cell, xi = (1 - albedo) tau eta; counts |eta| >= 1
// (or non-finite eta) into *bad.
hipError_t launch_dich_xi(int64_t C, const float *tau, const float *alb, const float *eta, float *xi, int *bad,
                          hipStream_t s);
// gacc: per-cell sums [3][C] (with eta, dichroic absorption: [4][C], the
// fourth the xi-derivative term)
hipError_t launch_gradchain(int64_t C, const float *tau, const float *alb, uint32_t flags,
                            const double *gacc, float *g_tau, float *g_alb, float *g_emis,
                            hipStream_t s, const float *eta = nullptr);

hipError_t launch_fill_f32(float *p, int64_t count, float v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s);

hipError_t launch_readout(const Geometry &g, const float *S, int edge, const int32_t *dirs,
                          int nout, float *out, hipStream_t s);
hipError_t launch_readout_adjoint(const Geometry &g, int edge, const int32_t *dirs, int nout,
                                  const float *gout, float *lam, hipStream_t s);
hipError_t launch_sums(const Geometry &g, const float *S, double *partial, int npart,
                       double *result, hipStream_t s);
hipError_t launch_maps(const Geometry &g, const float *S, float *I_mean, float *dop_mean,
                       hipStream_t s);

int sums_partials(const Geometry &g);

// Allocation-free totals: the partial sums live in a static device array.
// scratch_setup takes its address on `device` (which must be current) once
// per device; launch_sums_noalloc then writes the four float64 sums of S to
// result (device) through it.  Calls that overlap on one device share the
// array and race.
hipError_t scratch_setup(int device);
int scratch_partials_max();
hipError_t launch_sums_noalloc(const Geometry &g, int device, const float *S, double *result, hipStream_t s);

// LDS bytes of the fused launch the library will use (SIZE_MAX if none fits).
// three_d: the 3-D fused forward step (its direction weights in LDS too).
size_t step_lds_bytes(const Geometry &g, int prec, bool adjoint, bool dich = false, bool three_d = false);

}  // namespace rtl
