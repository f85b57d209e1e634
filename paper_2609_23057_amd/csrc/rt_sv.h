// Device launchers of the statevector emulation of the paper's one-step
// circuit (Sec. 2.1.2-2.1.8): a real float64 statevector over nq qubits,
// one array element per basis state (flat index bit q = qubit q).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rtl {

constexpr int kSvMaxAddr = 20;   // address qubits of a gate's angle table

// A real 2x2 gate between two basis values of the qubits in `mask` (one
// qubit: v0 = 0, v1 = the qubit's bit; two qubits: the Q <-> U pair of the
// Stokes register): for every basis state base whose mask bits are zero and
// whose control bits match ((base & cmask) == cval),
//   (a0, a1) = (psi[base | v0], psi[base | v1])
//   -> (u00 a0 + u01 a1, u10 a0 + u11 a1)
// with (u00, u01, u10, u11) = table[4 a .. 4 a + 3], a = sum_j bit(addr[j]) 2^j.
struct SvGate {
  uint64_t mask, v0, v1;
  uint64_t cmask, cval;
  int32_t nbits;       // qubits in mask (1 or 2)
  int32_t pos[2];      // their bit positions, ascending
  int32_t naddr;
  int32_t addr[kSvMaxAddr];
  const double *table;
  // mask qubits whose 1 half has never been written (an ancilla no launch
  // has acted on): that member of each pair is taken as zero, not read
  uint64_t zread;
  // filled by sv_launch_gate: the mask and control bits in ascending order;
  // threads enumerate only the states whose control bits match
  int32_t nfixed;
  int32_t fixed[24];
};
hipError_t sv_launch_gate(double *psi, int nq, const SvGate &g, hipStream_t s);

// Consecutive gates whose target qubits lie in one set of m <= 3 qubits
// (tq, ascending), applied in one pass: each thread loads the 2^m amplitudes
// that differ only in those qubits, applies the gates in order (for each, the
// pairs of its target within the set whose control qubits match, with the
// table entry of their address bits; the same products as sv_launch_gate,
// so the result is the same to the bit) and stores them.  Control qubits
// that every gate of the run shares with the same value (outside the target
// set: ccmask / ccval) are fixed, so the pass visits only those states.  A
// gate's local code: c in 0 .. m - 1 for a one-qubit gate on tq[c]; for the
// Q <-> U pair, 3 + 3 a + b with v0 on tq[a] and v1 on tq[b].
constexpr int kSvFuseMaxQ = 3;
constexpr int kSvFuseMaxGates = 8;
struct SvFusedGate {
  uint64_t cmask, cval;
  const double *table;
  int32_t naddr;
  int32_t addr[kSvMaxAddr];
  int32_t code;
};
struct SvFuse {
  int32_t m, ngates;
  int32_t tq[kSvFuseMaxQ];
  uint64_t ccmask, ccval;
  int32_t zlocal;   // local states with a never-written target qubit at 1: taken as zero, not read
  // filled by sv_launch_fused: the target and shared control qubits, ascending
  int32_t nfixed;
  int32_t fixed[kSvFuseMaxQ + 16];
  SvFusedGate g[kSvFuseMaxGates];
};
hipError_t sv_launch_fused(double *psi, int nq, const SvFuse &f, hipStream_t s);

// Controlled translation of the register bits [r0, r0 + qr) (Eq. 36-38 with
// the escape marker of Sec. 2.1.7): for live states (sl bit 0), d_out = k
// (bits [d0, d0 + qd)) and branch bit b, the translation is t = base[k] + b;
// on an absorbing axis a state whose target lies outside is marked escaped
// (its escape bit flipped) instead, and the unmarked states translate
// modulo 2^qr.  out[o] = in[src(o)] (a permutation; in and out distinct).
struct SvShift {
  int32_t r0, qr, ebit, abit, slbit, d0, qd, periodic;
  const int32_t *base;   // [2^qd]
  // qubits (none of them the escape marker) at which every amplitude of
  // `in` with a 1 is zero: such outputs are written as zero without a read
  uint64_t zmask;
  // the escape marker has never been set: a source with it at 1 is zero
  // (never written), not read
  int32_t ezero;
};
hipError_t sv_launch_shift(const double *in, double *out, int nq, const SvShift &t, hipStream_t s);

hipError_t sv_launch_zero(double *psi, uint64_t count, hipStream_t s);

// Sum of squares of a[0 .. na) and b[0 .. nb) into *result (device), via
// `partial` (device, sv_norm_partials() doubles).
int sv_norm_partials();
hipError_t sv_launch_norm2(const double *a, uint64_t na, const double *b, uint64_t nb, double *partial,
                           double *result, hipStream_t s);

// Amplitude encoding (Eq. 4): psi (zeroed) receives S[d][st][y][x] / norm at
// (st, sl = 0, d_in = d_out = d, y, x) and J[d][st][y][x] / norm at sl = 1,
// norm = sqrt(*norm2); data index ((((st 2 + sl) nd + d_in) nd + d_out) ny + y) nx + x.
// The same encoding written over the whole data block (the 2^ndata states
// with every ancilla at 0, zeros included), for a vector that is not zeroed
// first.
hipError_t sv_launch_encode_block(double *psi, const double *S, const double *J, int n, int nd, int ny, int nx,
                                  const double *norm2, hipStream_t s);
hipError_t sv_launch_encode(double *psi, const double *S, const double *J, int n, int nd, int ny, int nx,
                            const double *norm2, hipStream_t s);

// Decoding (Sec. 2.1.8): S'[k][st][y][x] = (sum over d_in of psi at (st,
// sl = 0, d_in, d_out = k, y, x)) * (scale2 * sqrt(*norm2)).
hipError_t sv_launch_decode(const double *psi, double *S, int n, int nd, int ny, int nx, double scale2,
                            const double *norm2, hipStream_t s);

}  // namespace rtl
