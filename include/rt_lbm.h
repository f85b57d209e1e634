/*
 * rt_lbm.h -- C ABI of the MI355X polarized lattice-Boltzmann radiative-transfer solver.
 *
 * The solver advances Stokes populations S[d][s][y][x] (direction d, Stokes
 * component s in I,Q,U,V, lattice row y, column x) one time step at a time:
 * emission, Beer-Lambert absorption, scattering through the rotated 4x4
 * phase matrix and bilinear streaming along the lattice displacement of each
 * direction (paper: Sec. 2.1.1 Eq. 2; operator chain Eq. 5 with states Eq. 8,
 * 10, 32, 39; emission Eq. 6; absorption Sec. 2.1.4; scattering Eq. 11-17 and
 * 21-30; streaming Eq. 33-39; boundaries Sec. 2.1.7).  The library also
 * provides the edge readout, diagnostic maps and the adjoint of a time-stepped
 * run with respect to per-cell extinction, albedo and emission.
 *
 * Conventions shared by every call
 *  - Memory: every d_* pointer is device memory owned by the caller (for
 *    example a torch tensor's data_ptr()), float32 unless stated.  It must stay
 *    valid until the work queued on the context's stream has finished.  h_*
 *    pointers are host memory read (or written) during the call only.  The
 *    library allocates no device memory: all persistent device data lives in
 *    the caller's workspace, whose size rt_workspace_bytes() returns (and a
 *    32 KiB static array per device, the scratch of rt_totals_noalloc).
 *  - State layout: S[d][s][y][x], d = i_zen * n_az + j_az, s = 0..3 (I,Q,U,V),
 *    x fastest; 4 * n * nx * ny floats, where n = n_zen * n_az.
 *  - Stokes vectors of direction d are referred to its meridian frame
 *    (e_theta, e_phi), polar axis +z.
 *  - Asynchrony: all calls that take a context enqueue on the context's
 *    stream and return without waiting, except where an h_* output is
 *    written (those synchronise the stream).
 *  - Errors: every call returns an rt_status; a message is available from
 *    rt_last_error(ctx) (or rt_last_error(NULL) for calls without a context).
 *    No call throws.  A context is used by one host thread at a time.
 */
#ifndef RT_LBM_H
#define RT_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx rt_ctx;

typedef enum {
  RT_OK = 0,
  RT_EINVAL = 1,        /* null pointer, bad size or enum, NaN/Inf, albedo outside [0,1], tau < 0 */
  RT_ERANGE = 2,        /* survival 1 - tau_sca < 0 (Eq. 31), |l| > 1, non-finite totals */
  RT_ESTATE = 3,        /* call order misuse, e.g. stepping before rt_set_medium */
  RT_ENOMEM = 4,        /* workspace or scratch buffer smaller than required */
  RT_EDEVICE = 5,       /* a HIP runtime error */
  RT_EUNSUPPORTED = 6   /* device is not gfx950, or an unsupported option combination */
} rt_status;

/* Arithmetic of the direction-pair contraction (the collision).  The state is
 * always float32; streaming, emission, absorption and the survival term are
 * always float32.  RT_FP32 uses float32 matrix cores.  RT_BF16 rounds the
 * state operand to bf16 and holds the collision matrix as a bf16 high part
 * plus a bf16 low part (two products; one bf16 rounding of the matrix would
 * bias the polarisation every step in the same direction).  RT_FP16 rounds
 * both operands to fp16 (a per-cell power-of-two scale of the state and a
 * global one of the matrix).  RT_BF16X3 splits both operands into bf16 high
 * and low parts and sums the three leading products.  All accumulate in
 * float32. */
typedef enum { RT_FP32 = 0, RT_BF16 = 1, RT_FP16 = 2, RT_BF16X3 = 3 } rt_precision;

/* Zenith nodes: equal-area cos(theta) midpoints arccos(1 - (2i+1)/n_zen)
 * (the reading of "uniformly distributed" pinned at n_zen = 2 by the DOP
 * table of Sec. 3.2.2), uniform theta (i+1) pi/(n_zen+1), or explicit degrees. */
typedef enum { RT_ZEN_EQUAL_AREA = 0, RT_ZEN_UNIFORM_THETA = 1, RT_ZEN_EXPLICIT = 2 } rt_zen_rule;

/* Lattice plane and displacement per step l(d) (Eq. 33):
 *   RT_PLANE_XY       l = courant * (k_x, k_y)   (horizontal plane)
 *   RT_PLANE_XZ       l = courant * (k_x, k_z)   (vertical plane, lattice y = altitude)
 *   RT_PLANE_XY_D2Q9  each component of (cos phi, sin phi) rounded to -1, 0 or 1
 *                     (the D2Q9 velocities of Sec. 2.1); components within 1e-6
 *                     of +-1/2 are refused as ambiguous.
 *   RT_PLANE_3D       a three-dimensional nx x ny x nz lattice (z = altitude),
 *                     l = courant * (k_x, k_y, k_z): the pull of Eq. 34 along
 *                     all three axes (trilinear), the collision per cell as in
 *                     2-D (the paper's conclusions name the extension to three
 *                     dimensions).  States are [4n][nz][ny][nx], cell
 *                     c = (z ny + y) nx + x; per-cell fields are [nz][ny][nx].
 *                     Faces x-, x+, y-, y+ take bc[0..3], z-, z+ take bc_z[0..1];
 *                     a ghost outside in z takes its z face, else its y face,
 *                     else its x face.  rt_step, rt_run (with checkpoints),
 *                     rt_stream, rt_maps, rt_readout / rt_readout_adjoint /
 *                     rt_num_outgoing per face (edge = face 0..5),
 *                     rt_set_phase_mixture, rt_set_dichroism and rt_adjoint;
 *                     the batch returns RT_EUNSUPPORTED. */
typedef enum { RT_PLANE_XY = 0, RT_PLANE_XZ = 1, RT_PLANE_XY_D2Q9 = 2, RT_PLANE_3D = 3 } rt_plane;

/* Edges are numbered 0 = x-, 1 = x+, 2 = y-, 3 = y+.  Periodic is the
 * recycling boundary of Eq. 39 (both edges of an axis must be periodic or
 * neither); absorbing discards what leaves (Sec. 2.1.7); inflow supplies a
 * prescribed radiance per edge and direction to what enters. */
typedef enum { RT_BC_PERIODIC = 0, RT_BC_ABSORBING = 1, RT_BC_INFLOW = 2 } rt_bc;

/* Scalar phase function used in the Eq. 17 weights.  For the first three
 * kinds the polarisation part is the Rayleigh reduced matrix rotated into the
 * meridian frames (Eq. 13, 16), so HG and the mixture carry Rayleigh-shaped
 * P12/P33/P44 ratios.  HG(g) = (1-g^2)/(4 pi (1+g^2-2g cos)^1.5); the mixture
 * is mix_ray * Rayleigh + (1 - mix_ray) * HG(g).
 *
 * RT_PHASE_TABLE: a general scattering matrix (the full-Mueller
 * representation the paper's conclusions name as future work; Mie-type
 * particles with P12 and P34 != 0), tabulated against the scattering angle.
 * rt_problem.table holds n_table rows (theta_deg, a1, a2, a3, a4, b1, b2) of
 *     F = [[a1, b1, 0, 0], [b1, a2, 0, 0], [0, 0, a3, b2], [0, 0, -b2, a4]]
 * referred to the scattering plane (axes e_par = n x k and n = k_in x k_out
 * normalised; Q = |E_par|^2 - |E_n|^2, U = 2 Re(E_par E_n*),
 * V = 2 Im(E_par E_n*)), with theta strictly increasing from exactly 0 to
 * exactly 180 and every a1 > 0.  F is linear in theta between rows; it takes
 * the place of the Rayleigh matrix in Eq. 13 and a1 is the phase function
 * of Eq. 17.  Forward and backward, where the scattering plane is undefined
 * (n = e_phi of the incoming direction is used), F must not depend on it:
 * b1 = b2 = 0 and a3 = a2 at 0 degrees, a3 = -a2 at 180 degrees, to 1e-6 of
 * a1.  For one particle with amplitude functions S1 (perpendicular) and S2
 * (parallel): a1 = a2 = (|S1|^2+|S2|^2)/2, b1 = (|S2|^2-|S1|^2)/2,
 * a3 = a4 = Re(S2 S1*), b2 = -Im(S2 S1*). */
typedef enum { RT_PHASE_RAYLEIGH = 0, RT_PHASE_HG = 1, RT_PHASE_MIX = 2, RT_PHASE_TABLE = 3 } rt_phase;

/* Option flags. */
enum {
  RT_ABS_TAYLOR = 1u << 0,    /* absorption factor 1 - tau_abs instead of exp(-tau_abs) (Sec. 2.1.4) */
  RT_SCAT_EXP = 1u << 1,      /* survival exp(-tau_sca) instead of 1 - tau_sca (extension, not in the paper) */
  RT_FUSED_TAYLOR = 1u << 2,  /* literal Eq. 2: Y = (1-tau_ext) S + tau_sca M S + dt J */
  RT_RENORM_IROW = 1u << 3,   /* make sum_out of the Q,U -> I elements zero (exact conservation) */
  RT_SCALAR = 1u << 4,        /* intensity-only transport: keep the I -> I elements only */
  RT_PLAIN = 1u << 5          /* unfused reference path: separate stream and vector-ALU collision (RT_FP32 only) */
};

typedef struct {
  int32_t nx, ny;             /* lattice size, >= 1 each */
  int32_t n_zen, n_az;        /* direction grid, n = n_zen * n_az, 1 <= n <= 256 */
  int32_t zen_rule;           /* rt_zen_rule */
  const double *zen_deg;      /* host [n_zen] zenith angles in degrees for RT_ZEN_EXPLICIT, else NULL */
  double az_offset_deg;       /* azimuths phi_j = offset + 360 j / n_az (Table 1 uses 0 and 22.5) */
  int32_t plane;              /* rt_plane */
  double courant;             /* c dt / dx for RT_PLANE_XY / RT_PLANE_XZ */
  int32_t bc[4];              /* rt_bc per edge */
  int32_t phase;              /* rt_phase */
  double g;                   /* HG asymmetry for RT_PHASE_HG / RT_PHASE_MIX, |g| < 1 */
  double mix_ray;             /* Rayleigh fraction for RT_PHASE_MIX, in [0, 1] */
  double dt;                  /* time step multiplying the source J (Eq. 2, Eq. 8) */
  uint32_t flags;             /* RT_* option flags */
  int32_t precision;          /* rt_precision */
  int32_t n_table;            /* rows of `table` for RT_PHASE_TABLE (2 .. 65536), else ignored */
  const double *table;        /* host [n_table][7] for RT_PHASE_TABLE, else NULL; copied by rt_init */
  int32_t nz;                 /* layers of an RT_PLANE_3D lattice (>= 1); 0 or 1 for the 2-D planes */
  int32_t bc_z[2];            /* rt_bc of the z- and z+ faces (RT_PLANE_3D) */
  /* Explicit direction set (Sec. 2.1.1: the direction grid, its solid-angle
   * weights, and the lattice displacement of Eq. 33); each NULL keeps the
   * rule above.  Host arrays, copied by rt_init.  n = n_zen * n_az is the
   * number of directions either way; direction d keeps index d.
   *   dir_xyz     [n][3] unit vectors k (polar axis +z), none along the
   *               axis (no meridian plane there); replaces the zenith /
   *               azimuth grid; the meridian frame is e_phi along increasing
   *               azimuth, e_theta = e_phi x k
   *   dir_domega  [n] solid angles > 0, the weights of the Eq. 17
   *               normalisation (default 4 pi / n)
   *   shift       [n][2] ([n][3] on RT_PLANE_3D) displacement per step in
   *               cells, |l| <= 1 per axis (RT_ERANGE otherwise); replaces
   *               the plane rule and decides which directions leave through
   *               each edge (components within 1e-12 of an integer are that
   *               integer) */
  const double *dir_xyz;
  const double *dir_domega;
  const double *shift;
  /* Phase mixtures (rt_set_phase_mixture_k): how many further phase
   * functions the context can hold, 0 .. RT_MIX_MAX (0 counts as 1); the
   * workspace keeps their matrices and per-cell fractions. */
  int32_t mix_max;
} rt_problem;

/* Most further phase functions of one mixture (K = 1 + k <= 8 in all). */
#define RT_MIX_MAX 7

/* ---- host-only helpers (no device needed) ------------------------------ */

/* Checks a problem description; RT_OK or the error code with a message. */
rt_status rt_validate(const rt_problem *p);

/* Bytes of device workspace rt_init needs for p (0 if p is invalid).  About
 * 2 state buffers plus 2 adjoint buffers plus O(n^2 + cells) of tables. */
size_t rt_workspace_bytes(const rt_problem *p);

/* Bytes of one state S (4 * n * nx * ny floats, times nz on a 3-D lattice). */
size_t rt_state_bytes(const rt_problem *p);

/* Direction set and operators in float64, as the library builds them.
 *   h_dirs  [n][6] or NULL: theta, phi (radians), dOmega, l_x, l_y, outgoing
 *           edge mask (bit e set when direction d leaves through edge e)
 *   h_M     [4n][4n] or NULL: collision matrix, row 4*d_out+s_out, column
 *           4*d_in+s_in: the Eq. 17 weight times the Rayleigh Mueller matrix
 *           of the pair normalised to its I->I element (Eq. 13, 16, 25/30),
 *           built from the dipole field projection in the meridian frames. */
rt_status rt_describe(const rt_problem *p, double *h_dirs, double *h_M);

/* Number of directions leaving through `edge` (the readout width; on an
 * RT_PLANE_3D lattice `edge` is a face 0..5 and z faces count l_z). */
int32_t rt_num_outgoing(const rt_problem *p, int32_t edge);

/* ---- context ------------------------------------------------------------- */

/* Builds, in float64 on the host, what the problem statement fixes before
 * time stepping: the direction set and its solid angles (Sec. 2.1.1), the
 * lattice displacement of every direction (Eq. 33), the collision matrix of
 * Eq. 17 from the rotated phase matrix (Eq. 13-16, 21-22; the direction-pair
 * sum of Eq. 25/30) and the streaming taps (Eq. 34); uploads the tables into
 * d_ws (caller-owned, ws_bytes >= rt_workspace_bytes(p)) on `stream` (a
 * hipStream_t, NULL = default stream) and returns a context in *out
 * (owned by the library until rt_destroy).  Synchronises the stream.
 * Errors: those of rt_validate; RT_EINVAL for a NULL out or workspace,
 * RT_ENOMEM if ws_bytes is too small, RT_EUNSUPPORTED if the current device
 * is not gfx950 or the problem does not fit the fused kernels, RT_EDEVICE
 * for a HIP failure. */
rt_status rt_init(const rt_problem *p, void *d_ws, size_t ws_bytes, void *stream, rt_ctx **out);

/* Per-cell medium, [ny][nx] each: d_tau = per-step extinction optical depth
 * k_ext * dt (>= 0), d_albedo = k_scat / k_ext in [0, 1], d_emis = emission
 * amplitude eps.  The source of direction d is J = eps * h_jprof[d][0..3]
 * (host [n][4]).  h_inflow (host [4][n][4] or NULL = zero; [6][n][4] faces
 * x-, x+, y-, y+, z-, z+ on an RT_PLANE_3D lattice) is the radiance entering
 * through each inflow edge per direction.  The values are copied
 * into the workspace and the per-cell coefficients alpha = a s,
 * beta = a (1 - s) (a = absorption factor, s = survival, Eq. 11) are formed.
 * Validation needs the values on the host, so this call synchronises the
 * stream; RT_ERANGE if some cell has 1 - tau_sca < 0 (Eq. 31). */
rt_status rt_set_medium(rt_ctx *c, const float *d_tau, const float *d_albedo, const float *d_emis,
                        const float *h_jprof, const float *h_inflow);

/* Inflow radiance per edge cell of a 2-D lattice (the boundary sources of
 * the problem statement; Sec. 2.1.7 edges with a prescribed radiance):
 * d_inflow is device float32 [2 nx + 2 ny][n][4], the cells of the x- edge
 * (y = 0 .. ny-1), then the x+ edge (y), the y- edge (x = 0 .. nx-1) and the
 * y+ edge (x), each with the Stokes vector entering in every direction; it
 * is copied (the caller keeps ownership).  A tap of the pull (Eq. 34) that
 * falls outside the lattice reads the edge it crossed (a y edge before an x
 * edge) at the cell it lies beyond: its x on a y edge, clamped to the
 * lattice at the corners, its y on an x edge.  Only edges of kind
 * RT_BC_INFLOW use their cells' values (the others stay zero).  Replaces the
 * uniform radiance rt_set_medium set; a later rt_set_medium replaces it in
 * turn.  Synchronises the stream (the values are checked).  Errors:
 * RT_EINVAL for NULL or a non-finite value, RT_ESTATE before rt_set_medium,
 * RT_EUNSUPPORTED on an RT_PLANE_3D lattice (whose faces take uniform
 * radiance from rt_set_medium). */
rt_status rt_set_inflow(rt_ctx *c, const float *d_inflow);

/* Per-cell mixture of two phase functions.  With it set, the scattered part
 * of the collision becomes beta ((1 - f) M X + f M2 X): M is the context's
 * collision matrix, M2 the one a problem with phase2 / g2 / mix_ray2 (same
 * meaning as rt_problem's phase / g / mix_ray; RT_PHASE_TABLE is not
 * accepted here) and otherwise the context's
 * own fields would build, each normalised as Eq. 17 prescribes, and f the
 * per-cell fraction d_frac (device [ny][nx] float32, values in [0, 1],
 * copied into the workspace).  Every later rt_step / rt_run uses it; phase2 < 0
 * removes it (d_frac is then ignored).  Validation reads f on the host, so
 * the call synchronises the stream.  Every precision carries it: M2 is
 * packed like M (bf16x3 with its own low parts; RT_FP16 at M's power-of-two
 * scale, which shares the unscale of the epilogue).  Errors: RT_EINVAL for an
 * invalid phase function or a NULL d_frac; RT_ERANGE if some f is outside
 * [0, 1] or not finite, or, for RT_FP16, if max |M2| at M's scale reaches the
 * fp16 range (more than 8 max |M|) (the mixture is then off); RT_EUNSUPPORTED while
 * dichroic absorption is set.  rt_adjoint carries the mixture (its step
 * contracts M^T and M2^T, packed here too, and blends them per cell);
 * rt_batch_run and rt_batch_adjoint carry the mixture of a batch channel. */
rt_status rt_set_phase_mixture(rt_ctx *c, int32_t phase2, double g2, double mix_ray2, const float *d_frac);

/* Per-cell mixture of K = 1 + k phase functions (the aerosol and cloud
 * mixtures of Sec. 4 with more than two components).  The scattered part of
 * the collision becomes beta ((1 - sum_j f_j) M X + sum_j f_j M_j X): M_j is
 * the collision matrix that phase[j] / g[j] / mix_ray[j] (host arrays [k],
 * same meaning as rt_problem's phase / g / mix_ray; not RT_PHASE_TABLE)
 * build with the context's other fields, and f_j the per-cell fractions
 * d_frac (device float32 [k][ny][nx], [k][nz][ny][nx] on a 3-D lattice,
 * copied into the workspace) with f_j >= 0 and sum_j f_j <= 1 in every cell;
 * M keeps the rest.  k = 0 removes the mixture (the other arguments are then
 * ignored); rt_set_phase_mixture(c, phase2, g2, mix_ray2, d_frac) is k = 1.
 * Every precision, rt_step / rt_run / rt_adjoint, the plain path, 3-D
 * lattices (on the two-launch step) and batch channels carry it as they
 * carry two components; each further matrix costs one more contraction per
 * step.  Synchronises
 * the stream (the fractions are checked on the host).  Errors: RT_EINVAL for
 * k < 0, k above the context's rt_problem.mix_max (0 counting as 1), NULL
 * arrays, or an invalid phase function; RT_ERANGE if a fraction is negative
 * or not finite, if the fractions of a cell sum past 1 (summed in double),
 * or, for RT_FP16, if a further matrix exceeds the fp16 range at M's scale
 * (the mixture is then off); RT_EUNSUPPORTED while dichroic absorption is
 * set. */
rt_status rt_set_phase_mixture_k(rt_ctx *c, int32_t k, const int32_t *phase, const double *g, const double *mix_ray,
                                 const float *d_frac);

/* Dichroic absorption (polarisation-dependent extinction, which the paper's
 * conclusions name as missing).  The absorption optical depth of direction d
 * in cell c becomes the matrix tau_abs K with K = [[1, eta w_d, 0, 0],
 * [eta w_d, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]] in the meridian axes,
 * w_d = sin^2 theta_d (particles aligned about z: no dichroism along z),
 * tau_abs = (1 - albedo) tau: the linear polarisations along e_theta (I + Q)
 * and e_phi (I - Q) are absorbed by exp(-tau_abs (1 +- eta w_d)), U and V by
 * exp(-tau_abs).  As the absorption it acts before the scattering.  d_eta is
 * a device [ny][nx] float32 field with |eta| < 1, copied into the workspace;
 * NULL removes it.  Later rt_step / rt_run use it, and rt_set_medium keeps it
 * in step with a new medium.  Synchronises the stream (eta is checked).
 * Every precision and RT_PLAIN carry it.  Errors: RT_EUNSUPPORTED with
 * RT_ABS_TAYLOR or RT_FUSED_TAYLOR, or while a phase mixture is set; RT_ERANGE if some |eta| >= 1 or eta is not finite
 * (dichroism is then off).  rt_adjoint carries it (eta held fixed: its step
 * applies the symmetric factor to alpha mu + beta nu and adds the derivative
 * through xi = tau_abs eta to the tau and albedo gradients); rt_batch_run and
 * rt_batch_adjoint carry it for a batch channel; rt_set_phase_mixture returns
 * RT_EUNSUPPORTED while it is set. */
rt_status rt_set_dichroism(rt_ctx *c, const float *d_eta);

/* Tuning of the 3-D lattice's fused step (RT_PLANE_3D; ignored otherwise).
 * With the RT_FP32 contraction, rt_run and rt_adjoint fuse the trilinear pull
 * of step t into the operand load of the collision of step t + 1 (as on a
 * 2-D lattice); the 16-bit contractions, RT_PLAIN, a phase mixture and
 * dichroic absorption step as collision then streaming, which is faster
 * there.  Its tiles are runs of cells along x within one row
 * (y, z), taken in blocks of `layers` layers with z fastest: the rows that
 * neighbouring tiles read overlap while they are still cached.  0 restores
 * the default (64); values above nz act as nz.  The result does not depend
 * on it.  RT_EINVAL for layers < 0. */
rt_status rt_set_layer_block(rt_ctx *c, int32_t layers);

/* Tuning of the 2-D fused steps' tile order: with tiles > 0 (and nx a
 * multiple of 64 tiles) the tiles walk vertical strips `tiles` tiles of 64
 * cells wide (tiles / 2 tiles of 32 cells), every row of a strip before the
 * next strip, instead of the lattice's row order; the rows of all 4n planes
 * that the tiles in flight on an XCD share with the next output rows then
 * stay in its L2.  By default the strips are 4 tiles wide where a state
 * exceeds 256 MiB (more than the last-level cache holds) and row order is
 * kept below; 0 sets row order.  The result does not depend on it.
 * RT_EINVAL for tiles < 0. */
rt_status rt_set_tile_strip(rt_ctx *c, int32_t tiles);

/* One time step of Sec. 2.1.1 (Eq. 2 split as the operator chain of Eq. 5):
 * emission X = S_in + dt J (Eq. 6/8), absorption and scattering
 * Y = alpha X + beta M X (Sec. 2.1.4-2.1.5, Eq. 11), streaming
 * S_out = L(Y) (Eq. 33-34, edges Sec. 2.1.7 / Eq. 39).  d_S_in and d_S_out
 * are device states [n][4][ny][nx] (rt_state_bytes each), caller-owned, not
 * overlapping.  Asynchronous.  RT_ESTATE before rt_set_medium, RT_EINVAL
 * for NULL or overlapping states. */
rt_status rt_step(rt_ctx *c, const float *d_S_in, float *d_S_out);

/* Streaming alone (Sec. 2.1.6, Eq. 33-34): d_out[p] = bilinear pull of
 * d_in[p] by the displacement of plane p's direction, with the context's
 * edges (periodic wrap, Eq. 39; absorbing edges give zero; inflow edges give
 * the radiance set by rt_set_medium).  Both fields are device [4n][ny][nx]
 * float32 (rt_state_bytes), caller-owned, and must not overlap.  Fields that
 * are 16-byte aligned with nx a multiple of 4 take the vectorised kernel;
 * the result is the same either way.  RT_ESTATE before rt_set_medium (the
 * inflow radiance lives there).  Asynchronous on the context's stream. */
rt_status rt_stream(rt_ctx *c, const float *d_in, float *d_out);

/* nsteps time steps of Sec. 2.1.1 (as rt_step) in place on d_S (S_0 in,
 * S_nsteps out); the streaming of one step is fused with the collision of
 * the next, so the state makes one HBM round trip per step.  If d_ckpt is
 * not NULL it receives S_{k*ckpt_every} in slot k = 0 ..
 * ceil(nsteps/ckpt_every)-1 (device, caller-owned, slots of rt_state_bytes
 * each), as rt_adjoint expects.  Asynchronous.  RT_ESTATE before
 * rt_set_medium, RT_EINVAL for nsteps < 0 or ckpt_every < 1 with d_ckpt. */
rt_status rt_run(rt_ctx *c, float *d_S, int32_t nsteps, float *d_ckpt, int32_t ckpt_every);

/* The radiance leaving the lattice (the boundary radiance maps of
 * Sec. 3.2, taken at an edge row as the paper's figures take the field):
 * Stokes vectors of the outgoing directions on one edge row/column,
 * d_out[e][k][4] (device, caller-owned), e along the edge (x for edges 2,3;
 * y for edges 0,1), k over the directions leaving through the edge in
 * increasing d.  If h_sums is not NULL it receives the float64 sums of I, Q,
 * U, V over the whole field (the conservation totals; synchronises;
 * RT_ERANGE if not finite). On an
 * RT_PLANE_3D lattice `edge` is a face 0..5 (x-, x+, y-, y+, z-, z+) and
 * d_out[e][k][4] runs over the face's cells e = a + na b: x faces (y, z),
 * y faces (x, z), z faces (x, y), the first index fastest. */
rt_status rt_readout(rt_ctx *c, const float *d_S, int32_t edge, float *d_out, double *h_sums);

/* Statevector emulation of the paper's quantum circuit for one time step
 * (Sec. 2.1.2-2.1.8), on the device in float64: the classical state and the
 * source are amplitude-encoded (Eq. 4) into the registers st (2 qubits), sl,
 * d_in, d_out (ceil(log2 n) each), y and x (log2 ny, log2 nx), with twelve
 * ancillas for q_d = 3 (q_d + 9 in general): the emission LCU I + X/2 + ZX/2
 * (Eq. 7, two ancillas), the absorption R_y dilation (Eq. 9), the selector of
 * survival and redistribution (Eq. 12, 31), the PREP_joint -> SELECT_RPR ->
 * PREP_joint^dagger routing over the outgoing direction (Eq. 25-30; route
 * register of q_d qubits) with each pair's rotation-phase-rotation operator
 * (Eq. 13, 21-24) and the phase matrix block-encoded through its eigenbasis
 * (Eq. 18-20, one ancilla), and bilinear streaming with one R_y ancilla and
 * one escape marker per axis (Eq. 34-38, Sec. 2.1.7).  Post-selecting every
 * ancilla on |0> and decoding with the known normalisation (Sec. 2.1.8)
 * gives the classical step (rt_step) to float64 round-off.  The collision
 * matrix's pair blocks are read as w R(sigma_out) Zt R(sigma_in) with
 * Zt = F / F_11 of the Rayleigh form; its eigenvalue 2 / (1 + cos^2) is
 * encoded at half scale, the factor restored through the selector's weights
 * (s, 2 (1 - s)) and a uniform 1 / max_c (2 - s(c)) in the absorption
 * rotation.  Emulated: 2-D lattices with power-of-two nx and ny, periodic or
 * absorbing edges, Rayleigh / HG / mixed phase weights, RT_ABS_TAYLOR and
 * RT_SCAT_EXP; RT_EUNSUPPORTED otherwise (3-D, inflow edges, tabulated
 * matrices, phase mixtures, dichroic absorption, RT_FUSED_TAYLOR).
 *
 * rt_sv_qubits: total and data qubits of the context's circuit.
 * rt_sv_workspace_bytes: device bytes rt_sv_step needs (two statevectors of
 *   2^nqubits float64, gate tables, the encoded source); 0 if not emulated
 *   (rt_last_error says why).
 * rt_sv_gate_count: gates (rotations, controlled X/Z, H and the Q-U
 *   rotations) and translations of one step, and (if not NULL) the
 *   statevector bytes their launches read and write, 8 per amplitude (a
 *   gate launched alone touches the pairs whose control qubits match; a
 *   fused pass or a translation the states its fixed qubits select;
 *   amplitudes known to be zero are written, not read).
 * rt_sv_set_fusion: consecutive gates whose target qubits lie within
 *   max_qubits qubits (0 .. 3; default 3) are applied in one pass over the
 *   statevector (each thread holds the 2^m amplitudes that differ in those
 *   qubits and applies the gates in order) where that moves fewer bytes than
 *   launching them one by one, and with max_qubits >= 1 every launch skips
 *   the amplitudes known to be zero (an ancilla no gate or translation has
 *   acted on yet is |0>: it becomes a control fixed to 0); 0 launches every
 *   gate alone over the whole vector.  The products on every nonzero
 *   amplitude are the same, so the result does not depend on it.  RT_EINVAL
 *   outside 0 .. 3.
 * rt_sv_launch_count: launches of gates, fused passes and translations one
 *   step makes with the current fusion setting.
 * rt_sv_step: one emulated step of the context's medium (rt_set_medium must
 *   have succeeded) from d_S_in to d_S_out (device float64 [n][4][ny][nx],
 *   caller-owned, may be the same array); d_work is the caller's workspace
 *   of at least rt_sv_workspace_bytes(); h_psucc (or NULL) receives the
 *   post-selection success probability.  Synchronises the stream.  Errors:
 *   RT_EINVAL (NULL), RT_ESTATE (no medium), RT_ENOMEM (workspace too
 *   small), RT_EUNSUPPORTED (see above). */
rt_status rt_sv_qubits(const rt_ctx *c, int32_t *nqubits, int32_t *ndata);
size_t rt_sv_workspace_bytes(const rt_ctx *c);
rt_status rt_sv_gate_count(const rt_ctx *c, int32_t *ngates, int32_t *nshifts, double *bytes_per_step);
rt_status rt_sv_set_fusion(rt_ctx *c, int32_t max_qubits);
rt_status rt_sv_launch_count(const rt_ctx *c, int32_t *nlaunches);
rt_status rt_sv_step(rt_ctx *c, void *d_work, size_t work_bytes, const double *d_S_in, double *d_S_out,
                     double *h_psucc);

/* For callers that cannot allocate device memory or call a synchronising
 * function (code under HIP graph capture, tight serving loops): the float64
 * sums of I, Q, U, V over the whole field, as rt_readout's h_sums computes
 * them, written to d_sums (device [4], caller-owned) asynchronously on the
 * context's stream.  The partial sums live in a static device array of the
 * library (4 x 1024 float64, 32 KiB per device, held until the process ends)
 * instead of the workspace; the call allocates nothing and does not
 * synchronise.  Every lattice fits (the partial count never exceeds 1024;
 * RT_ERANGE otherwise).  Calls on one device share that array: calls that
 * overlap in time on one device (different streams, or different threads)
 * race and must be ordered by the caller. */
rt_status rt_totals_noalloc(rt_ctx *c, const float *d_S, double *d_sums);

/* Direction-mean intensity and direction-mean degree of polarisation
 * sqrt(Q^2+U^2+V^2)/I (Sec. 3.2.1) per cell, [ny][nx] each. */
rt_status rt_maps(rt_ctx *c, const float *d_S, float *d_I_mean, float *d_dop_mean);

/* Transpose of rt_readout: d_lambdaT (a full state) is set to zero except the
 * edge entries, which receive d_gout[e][k][4]. */
rt_status rt_readout_adjoint(rt_ctx *c, int32_t edge, const float *d_gout, float *d_lambdaT);

/* Bytes of the segment buffer rt_adjoint needs for ckpt_every. */
size_t rt_adjoint_segment_bytes(const rt_problem *p, int32_t ckpt_every);

/* Gradients of a loss L(S_nsteps) with respect to the per-cell medium, given
 * d_lambdaT = dL/dS_nsteps, by reverse time stepping with checkpoints written
 * by rt_run (same nsteps and ckpt_every; recomputes each segment into d_seg).
 * Outputs [ny][nx]: d_g_tau = dL/dtau, d_g_albedo = dL/dalbedo, d_g_emis =
 * dL/deps; d_lambda0 (state, or NULL) = dL/dS_0.  Inflow radiances and the
 * emission profile are treated as constants; a phase mixture's fraction f is
 * held fixed too (its step transposes the mixed scattering).  The reverse
 * steps run on the fused matrix-core kernels (float32 for an RT_PLAIN
 * context), so n <= 128 is required: RT_EUNSUPPORTED otherwise (and if the
 * dichroic adjoint step's fourth per-cell sum would not fit the LDS). */
rt_status rt_adjoint(rt_ctx *c, int32_t nsteps, const float *d_ckpt, int32_t ckpt_every, float *d_seg,
                     const float *d_lambdaT, float *d_g_tau, float *d_g_albedo, float *d_g_emis,
                     float *d_lambda0);

/* ---- Spectral batch ------------------------------------------------------
 * Independent problems -- spectral channels, each with its own lattice,
 * direction grid, phase function and medium -- advanced together on one
 * stream.  A time step of all channels is one persistent kernel launch per
 * class of channels (below) over a work queue of (channel, tile) items: the
 * fused step of Sec. 2.1 (Eq. 5) and its adjoint, per channel exactly as
 * rt_run / rt_adjoint compute it.
 * With graph mode on, a run or adjoint is recorded into a HIP graph once and
 * replayed.  Requirements: every channel has the same precision and flags
 * (RT_PLAIN excluded) and 4n rounded up to a multiple of 32 is 32, 64, 128 or
 * 256 (n <= 64).  Per-channel arrays of device pointers are passed as host
 * arrays of nchan entries. */
typedef struct rt_batch rt_batch;

/* Workspace bytes of a batch: the channels' workspaces plus the work-queue
 * descriptors.  0 if some problem is invalid. */
size_t rt_batch_workspace_bytes(const rt_problem *probs, int32_t nchan);

/* Creates a batch of nchan channels, probs[i] describing channel i, on the
 * given stream; d_ws must hold rt_batch_workspace_bytes(probs, nchan) bytes
 * (256-byte aligned).  Sets up every channel as rt_init does (synchronises). */
rt_status rt_batch_init(const rt_problem *probs, int32_t nchan, void *d_ws, size_t ws_bytes, void *stream,
                        rt_batch **out);

/* Context of channel ch, owned by the batch (do not destroy it): for
 * rt_set_medium, rt_set_inflow, rt_set_phase_mixture(_k), rt_readout,
 * rt_set_dichroism, rt_maps, rt_readout_adjoint of that channel.  A channel
 * with a phase mixture (its problem's mix_max bounds the components) or with
 * dichroic absorption runs in the batch as alone, bit for bit (the dichroic
 * channels of a class in a launch of their own); rt_batch_run and
 * rt_batch_adjoint return RT_EUNSUPPORTED for a dichroic channel whose class,
 * at its block size, cannot hold the dichroic adjoint's fourth per-cell sum
 * in the LDS. */
rt_status rt_batch_channel(rt_batch *b, int32_t ch, rt_ctx **out);

/* rt_run for every channel: h_states[i] is channel i's state (updated in
 * place); h_ckpt is NULL or gives each channel's checkpoint buffer as in
 * rt_run. */
rt_status rt_batch_run(rt_batch *b, float *const *h_states, int32_t nsteps, float *const *h_ckpt,
                       int32_t ckpt_every);

/* rt_adjoint for every channel (checkpoints from rt_batch_run with the same
 * nsteps and ckpt_every; h_seg[i] holds rt_adjoint_segment_bytes of channel
 * i).  Outputs as rt_adjoint, without lambda_0. */
rt_status rt_batch_adjoint(rt_batch *b, int32_t nsteps, float *const *h_ckpt, int32_t ckpt_every,
                           float *const *h_seg, float *const *h_lambdaT, float *const *h_g_tau,
                           float *const *h_g_albedo, float *const *h_g_emis);

/* Channel classes of a batch and their launch shape (the tuning table).
 * Channels with the same number of 32-row tiles per direction set,
 * W = ceil(4n / 32), form a class; a batched step makes one persistent
 * launch per class, in blocks of `block_waves` waves that run
 * block_waves / W tiles of that class side by side (the paper's Sec. 2.1
 * step on every tile, unchanged).  rt_batch_init takes the block size of
 * each class from the library's tuning table (measured on the 64-channel
 * spectral workload); rt_batch_set_tuning replaces it for one class
 * (block_waves a power-of-two multiple of W, at most 8; RT_EINVAL
 * otherwise, RT_EUNSUPPORTED if it does not fit the LDS) and drops recorded
 * graphs.  Results do not depend on the block size (every tile computes the
 * same arithmetic).  rt_batch_num_classes / rt_batch_class report the
 * classes in increasing W (host outputs). */
rt_status rt_batch_num_classes(const rt_batch *b, int32_t *h_count);
rt_status rt_batch_class(const rt_batch *b, int32_t k, int32_t *h_waves_per_tile, int32_t *h_block_waves,
                         int32_t *h_nchan);
rt_status rt_batch_set_tuning(rt_batch *b, int32_t waves_per_tile, int32_t block_waves);

/* Temporal blocking of a batch: channels are taken in order into groups
 * whose working set (two states per channel in rt_batch_run, ckpt_every + 3
 * in rt_batch_adjoint) stays within `bytes`, and a run or adjoint completes
 * every time step of one group before it starts the next, so that a group's
 * states stay in the last-level cache from one step to the next; a channel
 * larger than the budget is a group of its own, and 0 puts all channels in
 * one group (every step of all channels before the next step).  The default
 * is 128 MiB (of the MI355X's 256 MiB last-level cache).  A group of one
 * channel runs that channel's own (single-problem) kernels.  Results do not
 * depend on it (the channels are independent).  Drops recorded graphs. */
rt_status rt_batch_set_cache_budget(rt_batch *b, size_t bytes);

/* Graph mode (0 off, 1 on).  On: rt_batch_run and rt_batch_adjoint record
 * their launches into a HIP graph the first time they see a set of arguments
 * and replay it while the arguments stay the same (one graph per entry
 * point; new arguments record anew).  The device memory named by the
 * arguments must then stay allocated until the batch is destroyed or the
 * mode is switched off. */
rt_status rt_batch_set_graph(rt_batch *b, int32_t enabled);

/* Waits for the batch's stream. */
rt_status rt_batch_synchronize(rt_batch *b);

/* Releases the batch, its channel contexts and graphs (not the caller's
 * memory). */
rt_status rt_batch_destroy(rt_batch *b);

/* Waits for the context's stream. */
rt_status rt_synchronize(rt_ctx *c);

/* Releases the context (not the caller's memory). */
rt_status rt_destroy(rt_ctx *c);

const char *rt_status_str(rt_status s);
const char *rt_last_error(const rt_ctx *c);

/* Message of the last failed batch call (NULL batch: the last failure of any call). */
const char *rt_batch_last_error(const rt_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* RT_LBM_H */
