// C ABI of the polarized LBM solver: contexts, workspace layout, time loops.
//
// The forward time loop keeps the post-collision field Y_t in two workspace
// buffers and streams it inside the next step's load (fused kernel), so one
// step reads and writes the state once:
//   Y_0 = collide(S_0);  Y_t = collide(L(Y_{t-1}));  S_T = L(Y_{T-1}).
// The adjoint replays the run backwards with square-root checkpointing:
// rt_run stores S_{kK}; for each segment in reverse the forward is recomputed
// into the caller's segment buffer and the fused adjoint kernel walks it back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rt_internal.h"
#include "rt_kernels.h"
#include "rt_sv.h"

using namespace rtl;

namespace {

thread_local std::string g_last_error;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  // byte offsets into the workspace
  size_t tables, tables_bytes;   // uploaded host tables (rows, taps, tiles, fragments, M)
  size_t taps, taps3, taps3_rev, ghost_zero, outdirs, MT;   // MT: float32 M transposed, for the plain path
  size_t tiles_fwd32, tiles_adj32, tiles_fwd, tiles_adj;
  size_t frag_fwd32, frag_adj32, frag_fwd, frag_fwd_lo, frag_adj, frag_adj_lo;
  size_t jrow, ghost, ghost3;     // set by rt_set_medium (ghost3: the 3-D faces)
  size_t mix_tiles, mix_frag, mix_frag_lo, mix_MT, frac;   // phase mixture (rt_set_phase_mixture)
  size_t mix_tiles_adj, mix_frag_adj, mix_frag_adj_lo;       // its transpose, for the adjoint
  size_t mix_tiles_bytes, mix_frag_bytes;   // per further matrix
  int mix_count;                             // further matrices the regions hold (rt_problem.mix_max, at least 1)
  size_t dich_eta, dich_xi, dich_w;   // dichroic absorption (rt_set_dichroism); 0 bytes if unsupported
  size_t tau, alb, emis, alpha, beta;
  size_t gacc, partial, sums, bad;
  size_t Ya, Yb, La, Lb;
  size_t total;
  int npart;
};

struct Packed {
  std::vector<TileRange> t_fwd32, t_adj32, t_fwd, t_adj;
  std::vector<uint8_t> f_fwd32, f_adj32, f_fwd, f_fwd_lo, f_adj, f_adj_lo;
  double a_scale = 1.0;
};

void pack_all(const HostPlan &hp, int prec, Packed *pk) {
  std::vector<TileRange> dummy;
  pack_fragments(hp, false, FRAG_F32, 1.0, false, &pk->t_fwd32, &pk->f_fwd32);
  pack_fragments(hp, true, FRAG_F32, 1.0, false, &pk->t_adj32, &pk->f_adj32);
  if (prec == RT_FP32) {
    pk->t_fwd = pk->t_fwd32;
    pk->t_adj = pk->t_adj32;
    return;
  }
  FragKind kind = prec == RT_FP16 ? FRAG_F16 : FRAG_BF16;
  double scale = 1.0;
  if (prec == RT_FP16) {
    double mx = 0.0;
    for (double v : hp.M) mx = std::max(mx, std::fabs(v));
    int e = 0;
    if (mx > 0) std::frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
    scale = std::ldexp(1.0, 13 - e);  // max |M| scale in [2^12, 2^13)
  }
  pk->a_scale = scale;
  pack_fragments(hp, false, kind, scale, false, &pk->t_fwd, &pk->f_fwd);
  pack_fragments(hp, true, kind, scale, false, &pk->t_adj, &pk->f_adj);
  if (prec == RT_BF16X3 || prec == RT_BF16) {
    pack_fragments(hp, false, FRAG_BF16, 1.0, true, &dummy, &pk->f_fwd_lo);
    pack_fragments(hp, true, FRAG_BF16, 1.0, true, &dummy, &pk->f_adj_lo);
  }
}

Layout make_layout(const HostPlan &hp, const Packed &pk, int prec, bool prec_flags_plain, int mix_max) {
  Layout L{};
  L.mix_count = std::max(1, mix_max);
  const size_t C = (size_t)hp.nx * hp.ny;
  const size_t state = C * 4 * hp.n * sizeof(float);
  const int ntile = hp.Rpad / kTileRows;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.tables = off;
  L.taps = take(hp.n * sizeof(DirTaps));
  L.taps3 = take(hp.n * sizeof(DirTaps3));
  L.taps3_rev = take(hp.n * sizeof(DirTaps3));
  L.ghost_zero = take(7 * hp.Rpad * sizeof(float));   // zeros: the reverse 3-D pull's ghosts
  L.outdirs = take(6 * hp.n * sizeof(int32_t));   // per edge (2-D) or face (3-D)
  L.MT = take((size_t)hp.R * hp.R * sizeof(float));
  L.tiles_fwd32 = take(ntile * sizeof(TileRange));
  L.tiles_adj32 = take(ntile * sizeof(TileRange));
  L.tiles_fwd = take(ntile * sizeof(TileRange));
  L.tiles_adj = take(ntile * sizeof(TileRange));
  L.frag_fwd32 = take(pk.f_fwd32.size());
  L.frag_adj32 = take(pk.f_adj32.size());
  L.frag_fwd = take(pk.f_fwd.size());
  L.frag_fwd_lo = take(pk.f_fwd_lo.size());
  L.frag_adj = take(pk.f_adj.size());
  L.frag_adj_lo = take(pk.f_adj_lo.size());
  L.tables_bytes = off - L.tables;
  L.jrow = take(hp.Rpad * sizeof(float));
  // 2-D ghost radiance, one row of Rpad floats per edge cell (x- edge y =
  // 0..ny-1, x+ edge, y- edge x = 0..nx-1, y+ edge) and a row of zeros; a
  // 3-D context keeps it zero (its fused kernels' taps stay inside) and has
  // one row per face in ghost3 (6 faces + zeros)
  L.ghost = take((size_t)(2 * ((size_t)hp.nx + hp.ny) + 1) * hp.Rpad * sizeof(float));
  L.ghost3 = take(7 * hp.Rpad * sizeof(float));
  // phase mixture, for each of mix_count further matrices: tile ranges and
  // dense A fragments of the matrix and of its transpose in the contraction
  // precision (float32 for the plain path, whose adjoint replays on the fused
  // float32 kernels), the plain path's float32 transpose, per-cell fraction
  {
    const size_t K1 = (size_t)L.mix_count;
    const bool mix_plain = prec_flags_plain;   // the plain path contracts a float32 M2^T on the ALUs
    const bool f32 = prec == RT_FP32 || mix_plain;
    const int kstep = f32 ? 8 : 16;
    L.mix_frag_bytes = ((size_t)ntile * ((hp.Rpad + kstep - 1) / kstep) + 1) * 64 * 16;
    L.mix_tiles_bytes = ntile * sizeof(TileRange);
    const size_t lo = (!f32 && (prec == RT_BF16X3 || prec == RT_BF16)) ? L.mix_frag_bytes : 0;
    L.mix_tiles = take(K1 * L.mix_tiles_bytes);
    L.mix_frag = take(K1 * L.mix_frag_bytes);
    L.mix_frag_lo = take(K1 * lo);
    L.mix_tiles_adj = take(K1 * L.mix_tiles_bytes);
    L.mix_frag_adj = take(K1 * L.mix_frag_bytes);
    L.mix_frag_adj_lo = take(K1 * lo);
    L.mix_MT = take(mix_plain ? K1 * hp.R * hp.R * sizeof(float) : 0);
    L.frac = take(K1 * C * sizeof(float));
    // dichroic absorption: per-cell eta and tau_abs * eta, per-direction sin^2 theta
    const bool dich = true;   // every precision (and the plain path)
    L.dich_eta = take(dich ? C * sizeof(float) : 0);
    L.dich_xi = take(dich ? C * sizeof(float) : 0);
    L.dich_w = take(dich ? hp.n * sizeof(float) : 0);
  }
  L.tau = take(C * sizeof(float));
  L.alb = take(C * sizeof(float));
  L.emis = take(C * sizeof(float));
  L.alpha = take(C * sizeof(float));
  L.beta = take(C * sizeof(float));
  L.gacc = take(4 * C * sizeof(double));   // adjoint per-cell sums (4: with dichroic absorption)
  Geometry g{(int64_t)C, hp.nx, hp.ny, 0, 0, hp.n, hp.R, hp.Rpad};
  L.npart = sums_partials(g);
  L.partial = take((size_t)L.npart * 4 * sizeof(double));
  L.sums = take(4 * sizeof(double));
  L.bad = take(sizeof(int));
  L.Ya = take(state);
  L.Yb = take(state);
  L.La = take(state);
  L.Lb = take(state);
  L.total = off;
  return L;
}

}  // namespace

// Tile order of the fused 3-D step: rows are taken in blocks of this many
// layers, the layer index fastest within a block, so that the source rows a
// tile shares with its neighbours in z (and, within a block, in y) are read
// again while they are in the XCD's L2 or the last-level cache.
constexpr int kLayerBlock = 64;

// Tile order of the 2-D fused steps: vertical strips of 4 tiles of 64 cells
// (2 tiles of 32 cells) where the state exceeds the 256 MiB last-level
// cache, row order below.  Measured against row order at 1024^2, n = 128
// (2.15 GB per state): bf16 2.35 -> 2.13 ms per step, bf16x3 3.08 -> 2.84,
// fp16 2.35 -> 2.23, fp32 5.21 -> 5.16.  A lattice row of all 4n planes is
// 2 MB there: in row order the tiles in flight on an XCD span whole rows,
// and the source rows they share with the next output rows leave its 4 MB
// L2 before they are read again.  At 512^2, n = 32 (134 MB, resident in the
// last-level cache) the bench pass is unchanged (893 against 897 ms).
constexpr int kTileStrip = 4;
constexpr size_t kStripStateBytes = 256u << 20;

struct rt_ctx {
  rt_problem prob{};
  std::vector<double> zen;
  std::vector<double> table;   // copy of a tabulated scattering matrix
  std::vector<double> dir_xyz, dir_domega, shift;   // copies of an explicit direction set
  HostPlan hp;
  Packed pk;
  Layout L{};
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  Geometry geo{};
  std::vector<uint8_t> host_tables;
  // host staging of the asynchronous uploads of rt_set_medium / rt_set_inflow
  // (kept here so that they outlive the copies): 2-D ghost table, emission
  // rows, 3-D face table
  std::vector<float> host_medium, host_jrow, host_ghost3;
  std::vector<float> host_dich_w;  // sin^2 theta per direction (staging)
  int nout[6] = {0, 0, 0, 0, 0, 0};
  bool medium_set = false;
  bool mixture = false;   // rt_set_phase_mixture(_k) succeeded
  int nmix = 0;           // its further matrices
  bool dichroic = false;  // rt_set_dichroism succeeded
  bool three_d = false;   // RT_PLANE_3D lattice
  Stream3Args s3{};       // its streaming arguments
  Stream3Args s3rev{};    // the transpose of its streaming (the adjoint's reverse pull)
  int zblk = kLayerBlock; // 3-D fused step: layers per block of its tile order
  int strip = -1;         // 2-D fused steps: strip width of the tile order in tiles (0: row order; -1: by size)
  int sv_fuse = kSvFuseMaxQ;  // statevector emulation: target qubits of a fused gate pass (0: none)
  int prec = 0;
  int cu_count = 256;
  int device = 0;     // the HIP device current at rt_init
  std::string err;

  template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
  rt_status fail(rt_status s, const std::string &m) {
    err = m;
    g_last_error = m;
    return s;
  }
  rt_status hip(hipError_t e, const char *where) {
    if (e == hipSuccess) return RT_OK;
    return fail(RT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
  StepArgs args(bool adjoint) const;
};

StepArgs rt_ctx::args(bool adjoint) const {
  StepArgs a{};
  a.geo = geo;
  a.taps = at<DirTaps>(L.taps);
  a.jrow = at<float>(L.jrow);
  a.ghost = at<float>(L.ghost);
  a.alpha = at<float>(L.alpha);
  a.beta = at<float>(L.beta);
  a.emis = at<float>(L.emis);
  const bool fused_taylor = (prob.flags & RT_FUSED_TAYLOR) != 0;
  a.dt_pre = fused_taylor ? 0.0f : (float)prob.dt;
  a.dt_post = fused_taylor ? (float)prob.dt : 0.0f;
  const bool f32 = prec == P_F32;
  a.frag = at<uint4>(adjoint ? (f32 ? L.frag_adj32 : L.frag_adj) : (f32 ? L.frag_fwd32 : L.frag_fwd));
  a.frag_lo = at<uint4>(adjoint ? L.frag_adj_lo : L.frag_fwd_lo);
  a.tiles = at<TileRange>(adjoint ? (f32 ? L.tiles_adj32 : L.tiles_adj)
                                  : (f32 ? L.tiles_fwd32 : L.tiles_fwd));
  a.a_scale_inv = (float)(1.0 / pk.a_scale);
  a.gacc = at<double>(L.gacc);
  if (mixture) {
    // the plain collision reads MT2; the fused kernels (also the plain
    // path's adjoint replay) the fragments
    if ((prob.flags & RT_PLAIN) && !adjoint) a.MT2 = at<float>(L.mix_MT);
    a.frag2 = at<uint4>(adjoint ? L.mix_frag_adj : L.mix_frag);
    a.frag2_lo = at<uint4>(adjoint ? L.mix_frag_adj_lo : L.mix_frag_lo);
    a.tiles2 = at<TileRange>(adjoint ? L.mix_tiles_adj : L.mix_tiles);
    a.frac = at<float>(L.frac);
    a.nmix = nmix;
    a.frag2_stride = (int64_t)(L.mix_frag_bytes / sizeof(uint4));
  }
  if (dichroic) {
    a.dich_xi = at<float>(L.dich_xi);
    a.dich_w = at<float>(L.dich_w);
  }
  // strip order where whole strips of whole tiles cover every row, for the
  // widest tiles (64 cells) and therefore for every tile width
  const size_t sbytes = (size_t)geo.C * 16 * geo.n;
  const int w = strip >= 0 ? strip : (sbytes > kStripStateBytes ? kTileStrip : 0);
  if (!three_d && w > 0 && geo.nx % (64 * w) == 0) a.strip = w;
  a.nt_out = sbytes > kStripStateBytes ? 1 : 0;
  if (three_d) {
    a.ny3 = s3.ny;
    a.nz = s3.nz;
    a.per_z = s3.per_z;
    a.zblk = std::max(1, std::min(zblk, s3.nz));
    a.taps3 = at<DirTaps3>(L.taps3);
  }
  return a;
}

namespace {

rt_status set_err(rt_status s, const std::string &m) {
  g_last_error = m;
  return s;
}

rt_status plan_for(const rt_problem *p, HostPlan *hp, Packed *pk, Layout *L, std::string *msg) {
  rt_status st = build_plan(p, hp, msg);
  if (st != RT_OK) return st;
  pack_all(*hp, p->precision, pk);
  *L = make_layout(*hp, *pk, p->precision, (p->flags & RT_PLAIN) != 0, p->mix_max);
  return RT_OK;
}

size_t state_elems(const rt_ctx *c) { return (size_t)c->geo.C * 4 * c->geo.n; }

}  // namespace

extern "C" {

const char *rt_status_str(rt_status s) {
  switch (s) {
    case RT_OK: return "RT_OK";
    case RT_EINVAL: return "RT_EINVAL";
    case RT_ERANGE: return "RT_ERANGE";
    case RT_ESTATE: return "RT_ESTATE";
    case RT_ENOMEM: return "RT_ENOMEM";
    case RT_EDEVICE: return "RT_EDEVICE";
    case RT_EUNSUPPORTED: return "RT_EUNSUPPORTED";
  }
  return "RT_UNKNOWN";
}

const char *rt_last_error(const rt_ctx *c) { return c ? c->err.c_str() : g_last_error.c_str(); }

rt_status rt_validate(const rt_problem *p) {
  HostPlan hp;
  std::string msg;
  rt_status st = build_plan(p, &hp, &msg);
  if (st != RT_OK) return set_err(st, msg);
  if (!(p->flags & RT_PLAIN) && hp.Rpad > 512)
    return set_err(RT_EUNSUPPORTED, "the fused matrix-core path supports n <= 128 (use RT_PLAIN)");
  g_last_error.clear();
  return RT_OK;
}

size_t rt_workspace_bytes(const rt_problem *p) {
  if (rt_validate(p) != RT_OK) return 0;
  HostPlan hp;
  Packed pk;
  Layout L;
  std::string msg;
  if (plan_for(p, &hp, &pk, &L, &msg) != RT_OK) return 0;
  return L.total;
}

size_t rt_state_bytes(const rt_problem *p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->n_zen < 1 || p->n_az < 1) return 0;
  const size_t layers = (p->plane == RT_PLANE_3D && p->nz > 1) ? (size_t)p->nz : 1;
  return (size_t)p->nx * p->ny * layers * p->n_zen * p->n_az * 4 * sizeof(float);
}

size_t rt_adjoint_segment_bytes(const rt_problem *p, int32_t ckpt_every) {
  if (ckpt_every < 1) return 0;
  const size_t k = ckpt_every > 1 ? (size_t)(ckpt_every - 1) : 1;
  return k * rt_state_bytes(p);
}

rt_status rt_describe(const rt_problem *p, double *h_dirs, double *h_M) {
  HostPlan hp;
  std::string msg;
  rt_status st = build_plan(p, &hp, &msg);
  if (st != RT_OK) return set_err(st, msg);
  if (h_dirs) {
    for (int d = 0; d < hp.n; ++d) {
      h_dirs[6 * d + 0] = hp.theta[d];
      h_dirs[6 * d + 1] = hp.phi[d];
      h_dirs[6 * d + 2] = hp.domega[d];
      h_dirs[6 * d + 3] = hp.lx[d];
      h_dirs[6 * d + 4] = hp.ly[d];
      h_dirs[6 * d + 5] = hp.outmask[d];
    }
  }
  if (h_M) std::memcpy(h_M, hp.M.data(), hp.M.size() * sizeof(double));
  return RT_OK;
}

int32_t rt_num_outgoing(const rt_problem *p, int32_t edge) {
  HostPlan hp;
  std::string msg;
  const int nedge = (p && p->plane == RT_PLANE_3D) ? 6 : 4;
  if (edge < 0 || edge >= nedge || build_plan(p, &hp, &msg) != RT_OK) return -1;
  int k = 0;
  for (int d = 0; d < hp.n; ++d) k += (hp.outmask[d] >> edge) & 1;
  return k;
}

rt_status rt_init(const rt_problem *p, void *d_ws, size_t ws_bytes, void *stream, rt_ctx **out) {
  if (!out) return set_err(RT_EINVAL, "out is NULL");
  *out = nullptr;
  rt_status st = rt_validate(p);
  if (st != RT_OK) return st;
  if (!d_ws) return set_err(RT_EINVAL, "workspace is NULL");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return set_err(RT_EDEVICE, "no HIP device");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_err(RT_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", need gfx950");

  rt_ctx *c = new rt_ctx();
  c->prob = *p;
  if (p->zen_rule == RT_ZEN_EXPLICIT) {
    c->zen.assign(p->zen_deg, p->zen_deg + p->n_zen);
    c->prob.zen_deg = c->zen.data();
  } else {
    c->prob.zen_deg = nullptr;
  }
  if (p->phase == RT_PHASE_TABLE) {
    c->table.assign(p->table, p->table + 7 * (size_t)p->n_table);
    c->prob.table = c->table.data();
  } else {
    c->prob.table = nullptr;
    c->prob.n_table = 0;
  }
  {
    // explicit direction set: the context keeps its own copies
    const size_t n = (size_t)p->n_zen * p->n_az;
    const size_t dim = p->plane == RT_PLANE_3D ? 3 : 2;
    auto keep = [](const double *src, size_t count, std::vector<double> &v) -> const double * {
      if (!src) return nullptr;
      v.assign(src, src + count);
      return v.data();
    };
    c->prob.dir_xyz = keep(p->dir_xyz, 3 * n, c->dir_xyz);
    c->prob.dir_domega = keep(p->dir_domega, n, c->dir_domega);
    c->prob.shift = keep(p->shift, dim * n, c->shift);
  }
  std::string msg;
  st = plan_for(&c->prob, &c->hp, &c->pk, &c->L, &msg);
  if (st != RT_OK) {
    delete c;
    return set_err(st, msg);
  }
  if (ws_bytes < c->L.total) {
    delete c;
    return set_err(RT_ENOMEM, "workspace smaller than rt_workspace_bytes()");
  }
  c->ws = static_cast<char *>(d_ws);
  c->stream = static_cast<hipStream_t>(stream);
  c->prec = p->precision;
  const HostPlan &hp = c->hp;
  c->geo = Geometry{(int64_t)hp.nx * hp.ny, hp.nx, hp.ny, p->bc[0] == RT_BC_PERIODIC,
                    p->bc[2] == RT_BC_PERIODIC, hp.n, hp.R, hp.Rpad};

  // the fused kernels must fit the LDS budget
  const size_t lds_max = 160 * 1024;
  if (!(p->flags & RT_PLAIN) && (step_lds_bytes(c->geo, c->prec, false) > lds_max ||
                                 step_lds_bytes(c->geo, c->prec, true) > lds_max)) {
    delete c;
    return set_err(RT_EUNSUPPORTED, "problem does not fit the fused kernel's LDS budget");
  }
  c->cu_count = prop.multiProcessorCount;
  c->device = dev;
  // the static scratch of rt_totals_noalloc: its address on this device, once
  if (hipError_t e = scratch_setup(dev); e != hipSuccess) {
    delete c;
    return set_err(RT_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  }

  // host tables
  std::vector<uint8_t> &tb = c->host_tables;
  tb.assign(c->L.tables_bytes, 0);
  auto put = [&](size_t off, const void *src, size_t bytes) {
    if (bytes) std::memcpy(tb.data() + (off - c->L.tables), src, bytes);
  };
  std::vector<DirTaps> taps(hp.n);
  const bool is3d = p->plane == RT_PLANE_3D;
  for (int d = 0; d < hp.n; ++d) {
    // a 3-D lattice streams with its own kernel; the fused kernels see the
    // identity pull there (the adjoint kernel reads the reverse-pulled field)
    const double lxd = is3d ? 0.0 : hp.lx[d], lyd = is3d ? 0.0 : hp.ly[d];
    const double fx0 = std::floor(lxd), fy0 = std::floor(lyd);
    const double fx = lxd - fx0, fy = lyd - fy0;
    const double wx0 = 1.0 - fx, wx1 = fx, wy0 = 1.0 - fy, wy1 = fy;
    taps[d] = DirTaps{(int32_t)fx0, (int32_t)fy0, (float)wx0, (float)wx1, (float)wy0, (float)wy1,
                      (float)(wx0 * wy0), (float)(wx1 * wy0), (float)(wx0 * wy1), (float)(wx1 * wy1)};
  }
  put(c->L.taps, taps.data(), taps.size() * sizeof(DirTaps));
  std::vector<DirTaps3> taps3(hp.n), taps3_rev(hp.n);
  for (int d = 0; d < hp.n; ++d) {
    const double l[3] = {hp.lx[d], hp.ly[d], hp.lz[d]};
    double base[3], w[3][2];
    for (int a = 0; a < 3; ++a) {
      base[a] = std::floor(l[a]);
      const double f = l[a] - base[a];
      w[a][0] = 1.0 - f;
      w[a][1] = f;
    }
    DirTaps3 t{(int32_t)base[0], (int32_t)base[1], (int32_t)base[2], 0, {}};
    for (int b = 0; b < 8; ++b) t.w[b] = (float)(w[0][b & 1] * w[1][(b >> 1) & 1] * w[2][b >> 2]);
    taps3[d] = t;
    // transpose: in'(x) = sum_b w_b out(x + o_b) is the pull with base
    // offset -o0 - 1 along each axis and the two weights swapped; a base of
    // -2 (l = 1 exactly: its first weight is 0) becomes -1 with the weights
    // moved down, so that every base lies in [-1, 1] as the kernel assumes
    double rb[3], rw[3][2];
    for (int a = 0; a < 3; ++a) {
      rb[a] = -base[a] - 1.0;
      rw[a][0] = w[a][1];
      rw[a][1] = w[a][0];
      if (rb[a] < -1.0) {
        rb[a] += 1.0;
        rw[a][0] = rw[a][1];
        rw[a][1] = 0.0;
      }
    }
    DirTaps3 r{(int32_t)rb[0], (int32_t)rb[1], (int32_t)rb[2], 0, {}};
    for (int b = 0; b < 8; ++b) r.w[b] = (float)(rw[0][b & 1] * rw[1][(b >> 1) & 1] * rw[2][b >> 2]);
    taps3_rev[d] = r;
  }
  put(c->L.taps3, taps3.data(), taps3.size() * sizeof(DirTaps3));
  put(c->L.taps3_rev, taps3_rev.data(), taps3_rev.size() * sizeof(DirTaps3));
  if (p->plane == RT_PLANE_3D) {
    c->three_d = true;
    c->s3 = Stream3Args{c->geo.C, hp.nx, hp.ny_lattice, hp.nz, hp.n, hp.Rpad, p->bc[0] == RT_BC_PERIODIC,
                        p->bc[2] == RT_BC_PERIODIC, p->bc_z[0] == RT_BC_PERIODIC,
                        c->at<DirTaps3>(c->L.taps3), c->at<float>(c->L.ghost3)};
    c->s3rev = c->s3;
    c->s3rev.taps = c->at<DirTaps3>(c->L.taps3_rev);
    c->s3rev.ghost = c->at<float>(c->L.ghost_zero);
  }
  std::vector<int32_t> od(6 * hp.n, 0);
  for (int e = 0; e < (is3d ? 6 : 4); ++e) {
    int k = 0;
    for (int d = 0; d < hp.n; ++d)
      if ((hp.outmask[d] >> e) & 1) od[e * hp.n + k++] = d;
    c->nout[e] = k;
  }
  put(c->L.outdirs, od.data(), od.size() * sizeof(int32_t));
  // plain path: M^T in float32, row k (input row) holds M[r][k] for all output rows r
  std::vector<float> MT(hp.M.size());
  for (int r = 0; r < hp.R; ++r)
    for (int k = 0; k < hp.R; ++k) MT[(size_t)k * hp.R + r] = (float)hp.M[(size_t)r * hp.R + k];
  put(c->L.MT, MT.data(), MT.size() * sizeof(float));
  put(c->L.tiles_fwd32, c->pk.t_fwd32.data(), c->pk.t_fwd32.size() * sizeof(TileRange));
  put(c->L.tiles_adj32, c->pk.t_adj32.data(), c->pk.t_adj32.size() * sizeof(TileRange));
  put(c->L.tiles_fwd, c->pk.t_fwd.data(), c->pk.t_fwd.size() * sizeof(TileRange));
  put(c->L.tiles_adj, c->pk.t_adj.data(), c->pk.t_adj.size() * sizeof(TileRange));
  put(c->L.frag_fwd32, c->pk.f_fwd32.data(), c->pk.f_fwd32.size());
  put(c->L.frag_adj32, c->pk.f_adj32.data(), c->pk.f_adj32.size());
  put(c->L.frag_fwd, c->pk.f_fwd.data(), c->pk.f_fwd.size());
  put(c->L.frag_fwd_lo, c->pk.f_fwd_lo.data(), c->pk.f_fwd_lo.size());
  put(c->L.frag_adj, c->pk.f_adj.data(), c->pk.f_adj.size());
  put(c->L.frag_adj_lo, c->pk.f_adj_lo.data(), c->pk.f_adj_lo.size());
  st = c->hip(hipMemcpyAsync(c->ws + c->L.tables, tb.data(), tb.size(), hipMemcpyHostToDevice, c->stream),
              "upload tables");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "upload tables");
  if (st != RT_OK) {
    std::string m = c->err;
    delete c;
    return set_err(st, m);
  }
  *out = c;
  return RT_OK;
}

// First ghost row of a 2-D edge (rows run along the edge: y for the x
// edges, x for the y edges) and the row count of the table (the zero row last).
static int64_t edge_row0(const rt_ctx *c, int e) {
  const int64_t nx = c->geo.nx, ny = c->geo.ny;
  return e == 0 ? 0 : (e == 1 ? ny : (e == 2 ? 2 * ny : 2 * ny + nx));
}
static int64_t ghost_rows(const rt_ctx *c) { return 2 * ((int64_t)c->geo.nx + c->geo.ny) + 1; }

// Uploads the 2-D ghost table from per-edge-cell radiance src[cell][n][4]
// (cells in edge-row order); rows of edges that are not inflow stay zero.
static rt_status upload_ghost2d(rt_ctx *c, const float *src) {
  const int n = c->hp.n, Rp = c->hp.Rpad;
  std::vector<float> &hm = c->host_medium;
  hm.assign((size_t)ghost_rows(c) * Rp, 0.0f);
  for (int e = 0; e < 4; ++e) {
    if (c->prob.bc[e] != RT_BC_INFLOW) continue;
    const int64_t r0 = edge_row0(c, e), cnt = e < 2 ? c->geo.ny : c->geo.nx;
    for (int64_t k = 0; k < cnt; ++k)
      for (int d = 0; d < n; ++d)
        for (int s = 0; s < 4; ++s) {
          const float v = src ? src[((r0 + k) * n + d) * 4 + s] : 0.0f;
          if (!std::isfinite(v)) return c->fail(RT_EINVAL, "inflow radiance not finite");
          hm[(size_t)(r0 + k) * Rp + gemm_row(n, d, s)] = v;
        }
  }
  return c->hip(hipMemcpyAsync(c->ws + c->L.ghost, hm.data(), hm.size() * sizeof(float), hipMemcpyHostToDevice,
                               c->stream), "upload inflow");
}

rt_status rt_set_medium(rt_ctx *c, const float *d_tau, const float *d_albedo, const float *d_emis,
                        const float *h_jprof, const float *h_inflow) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_tau || !d_albedo || !d_emis || !h_jprof) return c->fail(RT_EINVAL, "NULL medium pointer");
  const HostPlan &hp = c->hp;
  const int n = hp.n, Rp = hp.Rpad;
  std::vector<float> &jrow = c->host_jrow, &g3 = c->host_ghost3;
  jrow.assign(Rp, 0.0f);
  g3.assign(7 * Rp, 0.0f);
  for (int d = 0; d < n; ++d)
    for (int s = 0; s < 4; ++s) {
      const float v = h_jprof[4 * d + s];
      if (!std::isfinite(v)) return c->fail(RT_EINVAL, "emission profile not finite");
      jrow[gemm_row(n, d, s)] = v;
    }
  rt_status st = RT_OK;
  if (c->three_d) {
    for (int e = 0; e < 6; ++e) {
      const int bc = e < 4 ? c->prob.bc[e] : c->prob.bc_z[e - 4];
      for (int d = 0; d < n; ++d)
        for (int s = 0; s < 4; ++s) {
          const float v = h_inflow ? h_inflow[(e * n + d) * 4 + s] : 0.0f;
          if (!std::isfinite(v)) return c->fail(RT_EINVAL, "inflow radiance not finite");
          g3[e * Rp + gemm_row(n, d, s)] = (bc == RT_BC_INFLOW) ? v : 0.0f;
        }
    }
    // the 2-D table of a 3-D context only ever supplies zeros (taps of weight
    // zero next to the lattice's first and last cells)
    c->host_medium.assign((size_t)ghost_rows(c) * Rp, 0.0f);
    st = c->hip(hipMemcpyAsync(c->ws + c->L.ghost, c->host_medium.data(), c->host_medium.size() * sizeof(float),
                               hipMemcpyHostToDevice, c->stream), "upload inflow");
  } else {
    // the radiance of each edge, the same at every cell of the edge
    std::vector<float> cells;
    if (h_inflow) {
      cells.assign((size_t)(ghost_rows(c) - 1) * n * 4, 0.0f);
      for (int e = 0; e < 4; ++e) {
        const int64_t r0 = edge_row0(c, e), cnt = e < 2 ? c->geo.ny : c->geo.nx;
        for (int64_t k = 0; k < cnt; ++k)
          std::memcpy(&cells[(size_t)(r0 + k) * n * 4], h_inflow + (size_t)e * n * 4, n * 4 * sizeof(float));
      }
    }
    st = upload_ghost2d(c, h_inflow ? cells.data() : nullptr);
  }
  static_assert(sizeof(float) == 4, "float");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(c->ws + c->L.jrow, jrow.data(), Rp * sizeof(float), hipMemcpyHostToDevice,
                               c->stream), "upload jprof");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(c->ws + c->L.ghost3, g3.data(), g3.size() * sizeof(float), hipMemcpyHostToDevice,
                               c->stream), "upload inflow");
  int *bad = c->at<int>(c->L.bad);
  if (st == RT_OK) st = c->hip(hipMemsetAsync(bad, 0, sizeof(int), c->stream), "clear counter");
  if (st == RT_OK)
    st = c->hip(launch_coef(c->geo.C, d_tau, d_albedo, d_emis, c->at<float>(c->L.tau), c->at<float>(c->L.alb),
                            c->at<float>(c->L.emis), c->at<float>(c->L.alpha), c->at<float>(c->L.beta),
                            c->prob.flags, bad, c->stream), "coef");
  int hbad = 0;
  if (st == RT_OK) st = c->hip(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "read counter");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "set_medium");
  if (st != RT_OK) return st;
  if (hbad) {
    c->medium_set = false;
    return c->fail(RT_ERANGE, std::to_string(hbad) +
                                  " cells have invalid tau/albedo/emission or a negative survival "
                                  "1 - tau_sca (or absorption factor)");
  }
  c->medium_set = true;
  if (c->dichroic) {
    // tau_abs * eta from the new medium (eta was validated when it was set)
    st = c->hip(launch_dich_xi(c->geo.C, c->at<float>(c->L.tau), c->at<float>(c->L.alb),
                               c->at<float>(c->L.dich_eta), c->at<float>(c->L.dich_xi), bad, c->stream),
                "dichroism");
    if (st != RT_OK) return st;
  }
  return RT_OK;
}

rt_status rt_set_inflow(rt_ctx *c, const float *d_inflow) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_inflow) return c->fail(RT_EINVAL, "NULL inflow pointer");
  if (c->three_d) return c->fail(RT_EUNSUPPORTED, "inflow per edge cell is for 2-D lattices (3-D faces: rt_set_medium)");
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_inflow before rt_set_medium");
  const size_t count = (size_t)(ghost_rows(c) - 1) * c->hp.n * 4;
  std::vector<float> h(count);
  rt_status st = c->hip(hipMemcpyAsync(h.data(), d_inflow, count * sizeof(float), hipMemcpyDeviceToHost, c->stream),
                        "read inflow");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "read inflow");
  if (st == RT_OK) st = upload_ghost2d(c, h.data());
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "upload inflow");
  return st;
}

rt_status rt_set_phase_mixture_k(rt_ctx *c, int32_t k, const int32_t *phase, const double *g, const double *mix_ray,
                                 const float *d_frac) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (k < 0) return c->fail(RT_EINVAL, "number of further phase functions < 0");
  if (k == 0) {
    c->mixture = false;
    c->nmix = 0;
    return RT_OK;
  }
  const Layout &L = c->L;
  if (k > L.mix_count)
    return c->fail(RT_EINVAL, std::to_string(k) + " further phase functions; the context holds " +
                                  std::to_string(L.mix_count) + " (rt_problem.mix_max)");
  if (!phase || !g || !mix_ray) return c->fail(RT_EINVAL, "NULL phase function arrays");
  if (!d_frac) return c->fail(RT_EINVAL, "NULL fraction pointer");
  if (c->dichroic) return c->fail(RT_EUNSUPPORTED, "a context takes a phase mixture or dichroic absorption, not both");
  const bool plain = (c->prob.flags & RT_PLAIN) != 0;
  // the contraction precision of the further matrices (float32 for the plain
  // path, whose adjoint replays on the fused float32 kernels); fp16 takes the
  // first matrix's power-of-two scale (all products share the epilogue's
  // unscale), so each must stay in the fp16 range at that scale
  const int pr = plain ? RT_FP32 : c->prob.precision;
  const bool has_lo = pr == RT_BF16X3 || pr == RT_BF16;
  const int ntile = c->hp.Rpad / kTileRows;
  const size_t fb = L.mix_frag_bytes, lob = has_lo ? fb : 0;
  std::vector<TileRange> tiles((size_t)k * ntile), tiles_adj((size_t)k * ntile);
  std::vector<uint8_t> frag((size_t)k * fb), frag_adj((size_t)k * fb), frag_lo((size_t)k * lob),
      frag_adj_lo((size_t)k * lob);
  const int R = c->hp.R;
  std::vector<float> MT(plain ? (size_t)k * R * R : 0);   // float32 M_j transposed, as the plain collision reads M
  for (int j = 0; j < k; ++j) {
    const std::string which = "further phase function " + std::to_string(j) + ": ";
    if (phase[j] == RT_PHASE_TABLE) return c->fail(RT_EINVAL, which + "a mixture component cannot be a table");
    // the same direction set and options, another scalar phase function
    // (Eq. 17 weights, Rayleigh polarisation part)
    rt_problem pj = c->prob;
    pj.phase = phase[j];
    pj.g = g[j];
    pj.mix_ray = mix_ray[j];
    pj.n_table = 0;
    pj.table = nullptr;
    HostPlan hpj;
    std::string msg;
    const rt_status st = build_plan(&pj, &hpj, &msg);
    if (st != RT_OK) return c->fail(st, which + msg);
    if (plain) {
      if (hpj.R != R) return c->fail(RT_EINVAL, which + "matrix size differs from the context's");
      float *dst = MT.data() + (size_t)j * R * R;
      for (int r = 0; r < R; ++r)
        for (int q = 0; q < R; ++q) dst[(size_t)q * R + r] = (float)hpj.M[(size_t)r * R + q];
    }
    if (pr == RT_FP16) {
      double mx = 0.0;
      for (double v : hpj.M) mx = std::max(mx, std::fabs(v));
      if (mx * c->pk.a_scale >= 65504.0) {
        c->mixture = false;
        return c->fail(RT_ERANGE, which + "exceeds the fp16 range at the first matrix's scale");
      }
    }
    const FragKind kind = pr == RT_FP32 ? FRAG_F32 : (pr == RT_FP16 ? FRAG_F16 : FRAG_BF16);
    const double sc = pr == RT_FP16 ? c->pk.a_scale : 1.0;
    std::vector<TileRange> t, ta, unused;
    std::vector<uint8_t> f, fa, fl, fal;
    pack_fragments(hpj, false, kind, sc, false, &t, &f);
    pack_fragments(hpj, true, kind, sc, false, &ta, &fa);
    if (has_lo) {
      pack_fragments(hpj, false, FRAG_BF16, 1.0, true, &unused, &fl);
      pack_fragments(hpj, true, FRAG_BF16, 1.0, true, &unused, &fal);
    }
    if (f.size() > fb || fa.size() > fb || t.size() > (size_t)ntile || ta.size() > (size_t)ntile ||
        fl.size() > lob || fal.size() > lob)
      return c->fail(RT_EINVAL, which + "fragments exceed their workspace region");
    std::copy(t.begin(), t.end(), tiles.begin() + (size_t)j * ntile);
    std::copy(ta.begin(), ta.end(), tiles_adj.begin() + (size_t)j * ntile);
    std::copy(f.begin(), f.end(), frag.begin() + (size_t)j * fb);
    std::copy(fa.begin(), fa.end(), frag_adj.begin() + (size_t)j * fb);
    std::copy(fl.begin(), fl.end(), frag_lo.begin() + (size_t)j * lob);
    std::copy(fal.begin(), fal.end(), frag_adj_lo.begin() + (size_t)j * lob);
  }
  c->mixture = false;
  c->nmix = 0;
  const size_t C = (size_t)c->geo.C;
  std::vector<float> hf((size_t)k * C);
  rt_status st = RT_OK;
  const struct { size_t off; const void *p; size_t n; } up[] = {
      {L.mix_MT, MT.data(), MT.size() * sizeof(float)},
      {L.mix_tiles, tiles.data(), tiles.size() * sizeof(TileRange)},
      {L.mix_tiles_adj, tiles_adj.data(), tiles_adj.size() * sizeof(TileRange)},
      {L.mix_frag, frag.data(), frag.size()},
      {L.mix_frag_adj, frag_adj.data(), frag_adj.size()},
      {L.mix_frag_lo, frag_lo.data(), frag_lo.size()},
      {L.mix_frag_adj_lo, frag_adj_lo.data(), frag_adj_lo.size()}};
  for (const auto &u : up)
    if (st == RT_OK && u.n)
      st = c->hip(hipMemcpyAsync(c->ws + u.off, u.p, u.n, hipMemcpyHostToDevice, c->stream),
                  "upload mixture matrices");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(c->ws + L.frac, d_frac, hf.size() * sizeof(float), hipMemcpyDeviceToDevice,
                               c->stream),
                "copy fractions");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(hf.data(), c->ws + L.frac, hf.size() * sizeof(float), hipMemcpyDeviceToHost,
                               c->stream),
                "read fractions");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "set_phase_mixture");
  if (st != RT_OK) return st;
  // every fraction finite and >= 0, their sum per cell <= 1 (in double; the
  // kernels' float32 sum in the same order then stays <= 1 as well)
  size_t bad = 0;
  for (size_t cell = 0; cell < C; ++cell) {
    double sum = 0.0;
    bool ok = true;
    for (int j = 0; j < k; ++j) {
      const float v = hf[(size_t)j * C + cell];
      ok = ok && std::isfinite(v) && v >= 0.0f;
      sum += v;
    }
    if (!ok || !(sum <= 1.0)) ++bad;
  }
  if (bad)
    return c->fail(RT_ERANGE, std::to_string(bad) + " cells have a mixture fraction below 0 or fractions summing past 1");
  c->nmix = k;
  c->mixture = true;
  return RT_OK;
}

rt_status rt_set_phase_mixture(rt_ctx *c, int32_t phase2, double g2, double mix_ray2, const float *d_frac) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (phase2 < 0) return rt_set_phase_mixture_k(c, 0, nullptr, nullptr, nullptr, nullptr);
  return rt_set_phase_mixture_k(c, 1, &phase2, &g2, &mix_ray2, d_frac);
}

rt_status rt_set_tile_strip(rt_ctx *c, int32_t tiles) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (tiles < 0) return c->fail(RT_EINVAL, "tiles < 0");
  c->strip = tiles;
  return RT_OK;
}

rt_status rt_set_layer_block(rt_ctx *c, int32_t layers) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (layers < 0) return c->fail(RT_EINVAL, "layers < 0");
  c->zblk = layers == 0 ? kLayerBlock : layers;
  return RT_OK;
}

rt_status rt_set_dichroism(rt_ctx *c, const float *d_eta) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_eta) {
    c->dichroic = false;
    return RT_OK;
  }
  if (c->prob.flags & (RT_ABS_TAYLOR | RT_FUSED_TAYLOR))
    return c->fail(RT_EUNSUPPORTED, "dichroic absorption is defined for Beer-Lambert absorption");
  if (c->mixture) return c->fail(RT_EUNSUPPORTED, "a context takes a phase mixture or dichroic absorption, not both");
  c->dichroic = false;
  const Layout &L = c->L;
  const int n = c->hp.n;
  std::vector<float> &hw = c->host_dich_w;
  hw.resize(n);
  for (int d = 0; d < n; ++d) {
    const double st = std::sin(c->hp.theta[d]);
    hw[d] = (float)(st * st);
  }
  const size_t C = (size_t)c->geo.C;
  int *bad = c->at<int>(L.bad);
  int hbad = 0;
  rt_status st = c->hip(hipMemcpyAsync(c->ws + L.dich_w, hw.data(), n * sizeof(float), hipMemcpyHostToDevice,
                                       c->stream), "upload direction factors");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(c->ws + L.dich_eta, d_eta, C * sizeof(float), hipMemcpyDeviceToDevice, c->stream),
                "copy eta");
  if (st == RT_OK) st = c->hip(hipMemsetAsync(bad, 0, sizeof(int), c->stream), "clear counter");
  // before rt_set_medium the coefficients are recomputed there; eta is checked either way
  if (st == RT_OK)
    st = c->hip(launch_dich_xi(c->geo.C, c->at<float>(L.tau), c->at<float>(L.alb), c->at<float>(L.dich_eta),
                               c->at<float>(L.dich_xi), bad, c->stream), "dichroism");
  if (st == RT_OK) st = c->hip(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream), "read counter");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "set_dichroism");
  if (st != RT_OK) return st;
  if (hbad) return c->fail(RT_ERANGE, std::to_string(hbad) + " cells have |eta| >= 1 or a non-finite eta");
  c->dichroic = true;
  return RT_OK;
}

static rt_status fwd_step(rt_ctx *c, const float *in, bool gather, float *out, float *s_out) {
  StepArgs a = c->args(false);
  a.in = in;
  a.out = out;
  a.s_out = s_out;
  return c->hip(launch_step_mfma(a, c->prec, gather, c->stream, c->cu_count), "step");
}

// The fused 3-D forward step (trilinear pull in the gather) serves float32
// contexts on the matrix cores without a phase mixture or dichroic
// absorption, within the LDS budget; the others step as collision then
// streaming.  At 256 x 256 x 64, n = 32, the fused step takes 2.78 ms against
// 2.85 ms for the two launches in float32, but 2.74 / 2.75 / 2.64 ms against
// 2.61 / 2.62 / 2.39 ms for bf16 / bf16x3 / fp16: its gather re-reads the
// source rows several times from beyond the L2 (the rows of all 4n planes
// around the tiles in flight on an XCD exceed its 4 MB), whatever the
// precision, which only the float32 contraction's longer collision hides.
static bool fused3_ok(const rt_ctx *c) {
  return c->three_d && c->prec == P_F32 && !(c->prob.flags & RT_PLAIN) && !c->mixture && !c->dichroic &&
         step_lds_bytes(c->geo, c->prec, false, false, true) <= 160 * 1024;
}

// Y_t = collision of L3(Y_{t-1}) + emission; s_out (optional) = S_t = L3(Y_{t-1}).
static rt_status fwd3_step(rt_ctx *c, const float *Yprev, float *Yout, float *s_out) {
  StepArgs a = c->args(false);
  a.ghost = c->at<float>(c->L.ghost3);
  a.in = Yprev;
  a.out = Yout;
  a.s_out = s_out;
  return c->hip(launch_step3_mfma(a, c->prec, c->stream, c->cu_count), "step3d");
}

// One step on a 3-D lattice: the collision of every cell (the fused kernel
// without its 2-D gather, or the plain collision), then the trilinear pull.
static rt_status step3d(rt_ctx *c, const float *S_in, float *S_out) {
  StepArgs a = c->args(false);
  float *Y = c->at<float>(c->L.Ya);
  rt_status st;
  if (c->prob.flags & RT_PLAIN)
    st = c->hip(launch_collide_valu(a, c->at<float>(c->L.MT), S_in, Y, c->stream), "collide");
  else
    st = fwd_step(c, S_in, false, Y, nullptr);
  if (st == RT_OK) st = c->hip(launch_stream3d(c->s3, Y, S_out, c->stream), "stream3d");
  return st;
}

static rt_status plain_step(rt_ctx *c, const float *S_in, float *S_out) {
  StepArgs a = c->args(false);
  float *Y = c->at<float>(c->L.Ya);
  rt_status st = c->hip(launch_collide_valu(a, c->at<float>(c->L.MT), S_in, Y, c->stream), "collide");
  if (st == RT_OK) st = c->hip(launch_stream(a, Y, S_out, c->stream), "stream");
  return st;
}

rt_status rt_step(rt_ctx *c, const float *d_S_in, float *d_S_out) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_S_in || !d_S_out) return c->fail(RT_EINVAL, "NULL state pointer");
  {
    const uintptr_t i0 = (uintptr_t)d_S_in, o0 = (uintptr_t)d_S_out;
    const uintptr_t bytes = (uintptr_t)state_elems(c) * sizeof(float);
    if (i0 < o0 + bytes && o0 < i0 + bytes) return c->fail(RT_EINVAL, "S_in and S_out overlap");
  }
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_medium has not succeeded");
  if (c->three_d) return step3d(c, d_S_in, d_S_out);
  if (c->prob.flags & RT_PLAIN) return plain_step(c, d_S_in, d_S_out);
  float *Y = c->at<float>(c->L.Ya);
  rt_status st = fwd_step(c, d_S_in, false, Y, nullptr);
  if (st == RT_OK) st = c->hip(launch_stream(c->args(false), Y, d_S_out, c->stream), "stream");
  return st;
}

rt_status rt_stream(rt_ctx *c, const float *d_in, float *d_out) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_in || !d_out) return c->fail(RT_EINVAL, "NULL field pointer");
  const size_t bytes = rt_state_bytes(&c->prob);
  const char *i0 = reinterpret_cast<const char *>(d_in), *o0 = reinterpret_cast<const char *>(d_out);
  if (i0 < o0 + bytes && o0 < i0 + bytes) return c->fail(RT_EINVAL, "d_in and d_out overlap");
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_medium has not succeeded");
  if (c->three_d) return c->hip(launch_stream3d(c->s3, d_in, d_out, c->stream), "stream3d");
  return c->hip(launch_stream(c->args(false), d_in, d_out, c->stream), "stream");
}

rt_status rt_run(rt_ctx *c, float *d_S, int32_t nsteps, float *d_ckpt, int32_t ckpt_every) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_S) return c->fail(RT_EINVAL, "NULL state pointer");
  if (nsteps < 0) return c->fail(RT_EINVAL, "nsteps < 0");
  if (d_ckpt && ckpt_every < 1) return c->fail(RT_EINVAL, "ckpt_every < 1");
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_medium has not succeeded");
  if (nsteps == 0) return RT_OK;
  const size_t sb = state_elems(c) * sizeof(float);
  auto slot = [&](int k) { return reinterpret_cast<float *>(reinterpret_cast<char *>(d_ckpt) + (size_t)k * sb); };
  rt_status st = RT_OK;
  if (fused3_ok(c)) {
    // 3-D: the streaming of step t fused into the collision of step t + 1
    float *Y[2] = {c->at<float>(c->L.Ya), c->at<float>(c->L.Yb)};
    if (d_ckpt) st = c->hip(hipMemcpyAsync(slot(0), d_S, sb, hipMemcpyDeviceToDevice, c->stream), "ckpt");
    if (st == RT_OK) st = fwd_step(c, d_S, false, Y[0], nullptr);
    for (int t = 1; t < nsteps && st == RT_OK; ++t) {
      float *s_out = (d_ckpt && t % ckpt_every == 0) ? slot(t / ckpt_every) : nullptr;
      st = fwd3_step(c, Y[(t - 1) & 1], Y[t & 1], s_out);
    }
    if (st == RT_OK) st = c->hip(launch_stream3d(c->s3, Y[(nsteps - 1) & 1], d_S, c->stream), "stream3d");
    return st;
  }
  if ((c->prob.flags & RT_PLAIN) || c->three_d) {
    // two passes per step (collision into the workspace, streaming back)
    for (int t = 0; t < nsteps && st == RT_OK; ++t) {
      if (d_ckpt && t % ckpt_every == 0)
        st = c->hip(hipMemcpyAsync(slot(t / ckpt_every), d_S, sb, hipMemcpyDeviceToDevice, c->stream), "ckpt");
      if (st == RT_OK) st = c->three_d ? step3d(c, d_S, d_S) : plain_step(c, d_S, d_S);
    }
    return st;
  }
  float *Y[2] = {c->at<float>(c->L.Ya), c->at<float>(c->L.Yb)};
  if (d_ckpt) st = c->hip(hipMemcpyAsync(slot(0), d_S, sb, hipMemcpyDeviceToDevice, c->stream), "ckpt");
  if (st == RT_OK) st = fwd_step(c, d_S, false, Y[0], nullptr);
  for (int t = 1; t < nsteps && st == RT_OK; ++t) {
    float *s_out = (d_ckpt && t % ckpt_every == 0) ? slot(t / ckpt_every) : nullptr;
    st = fwd_step(c, Y[(t - 1) & 1], true, Y[t & 1], s_out);
  }
  if (st == RT_OK) st = c->hip(launch_stream(c->args(false), Y[(nsteps - 1) & 1], d_S, c->stream), "stream");
  return st;
}

// Cells of face e of a 3-D lattice in readout order: x faces (y, z), y faces
// (x, z), z faces (x, y), the first index fastest.
static FaceMap face_map(const rt_ctx *c, int e) {
  const int64_t nx = c->s3.nx, ny = c->s3.ny, nz = c->s3.nz, layer = nx * ny;
  switch (e) {
    case 0: return FaceMap{0, nx, layer, (int32_t)ny, (int32_t)(ny * nz)};
    case 1: return FaceMap{nx - 1, nx, layer, (int32_t)ny, (int32_t)(ny * nz)};
    case 2: return FaceMap{0, 1, layer, (int32_t)nx, (int32_t)(nx * nz)};
    case 3: return FaceMap{(ny - 1) * nx, 1, layer, (int32_t)nx, (int32_t)(nx * nz)};
    case 4: return FaceMap{0, 1, nx, (int32_t)nx, (int32_t)(nx * ny)};
    default: return FaceMap{(nz - 1) * layer, 1, nx, (int32_t)nx, (int32_t)(nx * ny)};
  }
}

rt_status rt_readout(rt_ctx *c, const float *d_S, int32_t edge, float *d_out, double *h_sums) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_S) return c->fail(RT_EINVAL, "NULL state pointer");
  const int nedge = c->three_d ? 6 : 4;
  if (edge < 0 || edge >= nedge) return c->fail(RT_EINVAL, c->three_d ? "face must be 0..5" : "edge must be 0..3");
  rt_status st = RT_OK;
  const int32_t *dirs = c->at<int32_t>(c->L.outdirs) + edge * c->geo.n;
  if (d_out && c->three_d)
    st = c->hip(launch_readout_face(c->geo.C, face_map(c, edge), d_S, dirs, c->nout[edge], d_out, c->stream),
                "readout");
  else if (d_out)
    st = c->hip(launch_readout(c->geo, d_S, edge, dirs, c->nout[edge], d_out, c->stream), "readout");
  if (st == RT_OK && h_sums) {
    double *res = c->at<double>(c->L.sums);
    st = c->hip(launch_sums(c->geo, d_S, c->at<double>(c->L.partial), c->L.npart, res, c->stream), "sums");
    if (st == RT_OK) st = c->hip(hipMemcpyAsync(h_sums, res, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "sums");
    if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "sums");
    if (st == RT_OK)
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(h_sums[k])) return c->fail(RT_ERANGE, "non-finite Stokes totals");
  }
  return st;
}

rt_status rt_totals_noalloc(rt_ctx *c, const float *d_S, double *d_sums) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_S || !d_sums) return c->fail(RT_EINVAL, "NULL pointer");
  if (sums_partials(c->geo) > scratch_partials_max())
    return c->fail(RT_ERANGE, "the lattice needs more partial sums than the static scratch holds");
  return c->hip(launch_sums_noalloc(c->geo, c->device, d_S, d_sums, c->stream), "totals");
}

rt_status rt_maps(rt_ctx *c, const float *d_S, float *d_I_mean, float *d_dop_mean) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_S || !d_I_mean || !d_dop_mean) return c->fail(RT_EINVAL, "NULL pointer");
  return c->hip(launch_maps(c->geo, d_S, d_I_mean, d_dop_mean, c->stream), "maps");
}

rt_status rt_readout_adjoint(rt_ctx *c, int32_t edge, const float *d_gout, float *d_lambdaT) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_gout || !d_lambdaT) return c->fail(RT_EINVAL, "NULL pointer");
  const int nedge = c->three_d ? 6 : 4;
  if (edge < 0 || edge >= nedge) return c->fail(RT_EINVAL, c->three_d ? "face must be 0..5" : "edge must be 0..3");
  const int32_t *dirs = c->at<int32_t>(c->L.outdirs) + edge * c->geo.n;
  rt_status st = c->hip(launch_fill_f32(d_lambdaT, (int64_t)state_elems(c), 0.0f, c->stream), "fill");
  if (st == RT_OK && c->three_d)
    st = c->hip(launch_readout_face_adjoint(c->geo.C, face_map(c, edge), dirs, c->nout[edge], d_gout, d_lambdaT,
                                            c->stream), "readout adjoint");
  else if (st == RT_OK)
    st = c->hip(launch_readout_adjoint(c->geo, edge, dirs, c->nout[edge], d_gout, d_lambdaT, c->stream),
                "readout adjoint");
  return st;
}

rt_status rt_adjoint(rt_ctx *c, int32_t nsteps, const float *d_ckpt, int32_t ckpt_every, float *d_seg,
                     const float *d_lambdaT, float *d_g_tau, float *d_g_albedo, float *d_g_emis,
                     float *d_lambda0) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_ckpt || !d_lambdaT) return c->fail(RT_EINVAL, "NULL checkpoint or lambda_T");
  if (nsteps < 1 || ckpt_every < 1) return c->fail(RT_EINVAL, "nsteps and ckpt_every must be >= 1");
  if (ckpt_every > 1 && !d_seg) return c->fail(RT_EINVAL, "segment buffer is NULL");
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_medium has not succeeded");
  if (c->dichroic && step_lds_bytes(c->geo, (c->prob.flags & RT_PLAIN) ? P_F32 : c->prec, true, true) > 160 * 1024)
    return c->fail(RT_EUNSUPPORTED, "the dichroic adjoint step does not fit the LDS budget");
  if (c->geo.Rpad > 512)
    return c->fail(RT_EUNSUPPORTED, "the adjoint runs on the fused kernels, which support n <= 128");
  const int prec_save = c->prec;
  if (c->prob.flags & RT_PLAIN) c->prec = P_F32;  // the plain path replays on the fused float32 kernels
  const size_t sb = state_elems(c) * sizeof(float);
  auto ck = [&](int k) {
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(d_ckpt) + (size_t)k * sb);
  };
  auto seg = [&](int k) { return reinterpret_cast<float *>(reinterpret_cast<char *>(d_seg) + (size_t)k * sb); };
  rt_status st = c->hip(launch_fill_f64(c->at<double>(c->L.gacc), 4 * c->geo.C, 0.0, c->stream), "fill");
  float *Lb[2] = {c->at<float>(c->L.La), c->at<float>(c->L.Lb)};
  const float *lam_next = d_lambdaT;
  int flip = 0;
  const int nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  // 3-D lattice: the segments hold the states S_{t0+1} .. S_{t1-1}; each step
  // reverse-pulls lambda with the transposed trilinear taps into the
  // workspace, then runs the adjoint collision on it (identity 2-D taps) with
  // X read from the stored state
  for (int k = nseg - 1; c->three_d && k >= 0 && st == RT_OK; --k) {
    const int t0 = k * ckpt_every;
    const int t1 = std::min(nsteps, t0 + ckpt_every);
    if (t1 - t0 >= 2 && fused3_ok(c)) {
      // S_{t0+1} .. S_{t1-1} into the segment: the fused steps write S_t as
      // their streamed state, the last one is a streaming alone
      float *Y[2] = {c->at<float>(c->L.Ya), c->at<float>(c->L.Yb)};
      st = fwd_step(c, ck(k), false, Y[0], nullptr);
      for (int t = t0 + 1; t <= t1 - 2 && st == RT_OK; ++t)
        st = fwd3_step(c, Y[(t - 1 - t0) & 1], Y[(t - t0) & 1], seg(t - 1 - t0));
      if (st == RT_OK)
        st = c->hip(launch_stream3d(c->s3, Y[(t1 - 2 - t0) & 1], seg(t1 - 2 - t0), c->stream), "stream3d");
    } else if (t1 - t0 >= 2) {
      st = step3d(c, ck(k), seg(0));
      for (int t = t0 + 2; t <= t1 - 1 && st == RT_OK; ++t) st = step3d(c, seg(t - 2 - t0), seg(t - 1 - t0));
    }
    float *mu = c->at<float>(c->L.Ya);
    for (int t = t1 - 1; t >= t0 && st == RT_OK; --t) {
      st = c->hip(launch_stream3d(c->s3rev, lam_next, mu, c->stream), "reverse stream3d");
      if (st != RT_OK) break;
      StepArgs a = c->args(true);
      a.in = t > t0 ? seg(t - 1 - t0) : ck(k);
      a.lam_next = mu;
      a.out = Lb[flip];
      st = c->hip(launch_adjoint_mfma(a, c->prec, false, c->stream, c->cu_count), "adjoint");
      lam_next = Lb[flip];
      flip ^= 1;
    }
  }
  for (int k = nseg - 1; !c->three_d && k >= 0 && st == RT_OK; --k) {
    const int t0 = k * ckpt_every;
    const int t1 = std::min(nsteps, t0 + ckpt_every);
    // recompute Y_{t0} .. Y_{t1-2}
    if (t1 - t0 >= 2) {
      st = fwd_step(c, ck(k), false, seg(0), nullptr);
      for (int t = t0 + 1; t <= t1 - 2 && st == RT_OK; ++t)
        st = fwd_step(c, seg(t - 1 - t0), true, seg(t - t0), nullptr);
    }
    for (int t = t1 - 1; t >= t0 && st == RT_OK; --t) {
      StepArgs a = c->args(true);
      const bool gather = t > t0;
      a.in = gather ? seg(t - 1 - t0) : ck(k);
      a.lam_next = lam_next;
      a.out = Lb[flip];
      st = c->hip(launch_adjoint_mfma(a, c->prec, gather, c->stream, c->cu_count), "adjoint");
      lam_next = Lb[flip];
      flip ^= 1;
    }
  }
  if (st == RT_OK)
    st = c->hip(launch_gradchain(c->geo.C, c->at<float>(c->L.tau), c->at<float>(c->L.alb), c->prob.flags,
                                 c->at<double>(c->L.gacc), d_g_tau, d_g_albedo, d_g_emis, c->stream,
                                 c->dichroic ? c->at<float>(c->L.dich_eta) : nullptr), "gradchain");
  if (st == RT_OK && d_lambda0)
    st = c->hip(hipMemcpyAsync(d_lambda0, lam_next, sb, hipMemcpyDeviceToDevice, c->stream), "lambda0");
  c->prec = prec_save;
  return st;
}

// ------------------------------------------------- statevector emulation (circuit)

}  // extern "C"

namespace {

// Qubits of the emulated circuit (flat-index bits from the least significant):
// x, y, d_out, d_in, sl, st0, st1 (data), then em0, em1, abs, sel, route, pt,
// ax, ay, ex, ey (ancillas).  Stokes st = 2 st1 + st0.
struct SvLayout {
  int qx = 0, qy = 0, qd = 0, nd = 0, ndata = 0, nq = 0;
  int x0 = 0, y0 = 0, dout0 = 0, din0 = 0, sl = 0, st0 = 0, st1 = 0;
  int em0 = 0, em1 = 0, abs = 0, sel = 0, route0 = 0, pt = 0, ax = 0, ay = 0, ex = 0, ey = 0;
};

int log2_exact(int v) {
  int q = 0;
  while ((1 << q) < v) ++q;
  return (v >= 1 && (1 << q) == v) ? q : -1;
}

struct SvOp {
  bool shift = false;
  SvGate g{};
  size_t table_off = 0;   // doubles into the table region
  SvShift s{};
  int base_off = 0;       // int32 entries into the base table
};

struct SvCircuit {
  SvLayout L;
  std::vector<SvOp> ops;
  std::vector<double> tables;
  std::vector<int32_t> bases;
  std::vector<double> J;   // [n][4][ny][nx]: dt eps j (the sl = 1 sector)
  double lam_max = 1.0;
};

// Why a context cannot be emulated ("" if it can), and its layout.
std::string sv_check(const rt_ctx *c, SvLayout *L) {
  if (c->three_d) return "3-D lattices are not emulated";
  if (c->prob.flags & RT_FUSED_TAYLOR) return "the fused-Taylor form is not emulated";
  if (c->mixture || c->dichroic) return "phase mixtures and dichroic absorption are not emulated";
  for (int e = 0; e < 4; ++e)
    if (c->prob.bc[e] == RT_BC_INFLOW) return "inflow edges are not emulated";
  const HostPlan &hp = c->hp;
  L->qx = log2_exact(hp.nx);
  L->qy = log2_exact(hp.ny);
  if (L->qx < 0 || L->qy < 0) return "nx and ny must be powers of two";
  L->qd = 1;
  while ((1 << L->qd) < hp.n) ++L->qd;
  L->nd = 1 << L->qd;
  int pos = 0;
  auto take = [&](int w) { const int p0 = pos; pos += w; return p0; };
  L->x0 = take(L->qx);
  L->y0 = take(L->qy);
  L->dout0 = take(L->qd);
  L->din0 = take(L->qd);
  L->sl = take(1);
  L->st0 = take(1);
  L->st1 = take(1);
  L->ndata = pos;
  L->em0 = take(1);
  L->em1 = take(1);
  L->abs = take(1);
  L->sel = take(1);
  L->route0 = take(L->qd);
  L->pt = take(1);
  L->ax = take(1);
  L->ay = take(1);
  L->ex = take(1);
  L->ey = take(1);
  L->nq = pos;
  if (L->nq > 34) return "the statevector would exceed 2^34 amplitudes";
  return "";
}

// The circuit's gates and their tables for the context's operator and
// medium (host float64).  tau, alb, emis: the medium's float32 values.
std::string sv_compile(const rt_ctx *c, const std::vector<float> &tau, const std::vector<float> &alb,
                       const std::vector<float> &emis, SvCircuit *out) {
  SvCircuit &K = *out;
  std::string why = sv_check(c, &K.L);
  if (!why.empty()) return why;
  const SvLayout &L = K.L;
  const HostPlan &hp = c->hp;
  const int n = hp.n, nd = L.nd, nx = hp.nx, ny = hp.ny, C = nx * ny, R = hp.R;
  // --- per ordered pair (k <- d): w R(sigma_out) Zt R(sigma_in) with
  // Zt = [[1, b, 0, 0], [b, 1, 0, 0], [0, 0, g, 0], [0, 0, 0, g]], read off
  // the collision matrix and checked by rebuilding the block
  std::vector<double> w(nd * nd, 0.0), sin2(nd * nd, 0.0), sout2(nd * nd, 0.0), lam(nd * nd * 4, 0.0);
  auto rot = [](double a2, double v[4][4]) {   // R(psi) of Eq. 21 with a2 = 2 psi
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) v[i][j] = i == j ? 1.0 : 0.0;
    v[1][1] = v[2][2] = std::cos(a2);
    v[1][2] = std::sin(a2);
    v[2][1] = -std::sin(a2);
  };
  for (int d = 0; d < n; ++d)
    for (int k = 0; k < n; ++k) {
      double B[4][4];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) B[i][j] = hp.M[(size_t)(4 * k + i) * R + 4 * d + j];
      const double wk = B[0][0];
      double b = 0.0, g = 0.0, ai = 0.0, ao = 0.0;
      if (wk > 0.0) {
        b = -std::hypot(B[0][1], B[0][2]) / wk;
        g = B[3][3] / wk;
        if (std::fabs(b) > 1e-12) {
          ai = std::atan2(B[0][2] / (wk * b), B[0][1] / (wk * b));
          ao = std::atan2(-B[2][0] / (wk * b), B[1][0] / (wk * b));
        } else {
          ao = g > 0.0 ? std::atan2(B[1][2], B[1][1]) : std::atan2(-B[2][1], B[1][1]);
        }
        double Ri[4][4], Ro[4][4], Z[4][4] = {{1, b, 0, 0}, {b, 1, 0, 0}, {0, 0, g, 0}, {0, 0, 0, g}};
        rot(ai, Ri);
        rot(ao, Ro);
        double err = 0.0, mx = 1.0;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) {
            double v = 0.0;
            for (int p = 0; p < 4; ++p)
              for (int q = 0; q < 4; ++q) v += Ro[i][p] * Z[p][q] * Ri[q][j];
            err = std::max(err, std::fabs(wk * v - B[i][j]));
            mx = std::max(mx, std::fabs(B[i][j]));
          }
        if (err > 1e-12 * mx) return "the collision matrix is not of the rotation-phase-rotation form (tabulated matrices)";
      } else if (wk < 0.0) {
        return "negative scattering weight";
      }
      w[k * nd + d] = wk;
      sin2[d * nd + k] = ai;    // pair tables: index k + nd d (address d_out bits, then d_in bits)
      sout2[d * nd + k] = ao;
      const double ev[4] = {1.0 + b, 1.0 - b, g, g};   // by st after H on st0
      for (int st = 0; st < 4; ++st) lam[(st * nd + d) * nd + k] = ev[st];
    }
  // --- medium: alpha = a s, beta = a (1 - s) as the coefficient step forms
  // them, in float64
  const bool abs_taylor = (c->prob.flags & RT_ABS_TAYLOR) != 0, scat_exp = (c->prob.flags & RT_SCAT_EXP) != 0;
  std::vector<double> aabs(C), surv(C);
  double lam_max = 0.0;
  for (int i = 0; i < C; ++i) {
    const double t = tau[i], al = alb[i];
    const double t_sca = al * t, t_abs = (1.0 - al) * t;
    const double a = abs_taylor ? 1.0 - t_abs : std::exp(-t_abs);
    const double sv = scat_exp ? std::exp(-t_sca) : 1.0 - t_sca;
    const double alpha = a * sv, beta = a * (1.0 - sv);
    const double at = alpha + beta;
    const double s = at > 0.0 ? alpha / at : 1.0;
    if (at < 0.0 || at > 1.0 + 1e-15 || s < 0.0) return "coefficients outside 0 <= alpha, beta; alpha + beta <= 1";
    aabs[i] = at;
    surv[i] = s;
    lam_max = std::max(lam_max, 2.0 - s);
  }
  K.lam_max = lam_max;
  K.J.assign((size_t)n * 4 * C, 0.0);
  for (int d = 0; d < n; ++d)
    for (int st = 0; st < 4; ++st) {
      const size_t r = (size_t)gemm_row(n, d, st);
      const double j = r < c->host_jrow.size() ? (double)c->host_jrow[r] : 0.0;
      for (int i = 0; i < C; ++i) K.J[((size_t)d * 4 + st) * C + i] = (j * (double)emis[i]) * c->prob.dt;
    }
  // --- gate list
  K.ops.clear();
  K.tables.clear();
  K.bases.clear();
  auto bit = [](int b) { return 1ull << b; };
  // a gate on qubit q (or the Q <-> U pair when qu), controls, address bits
  // (table index bit j = addr[j]) and its table [2^naddr][4]
  auto gate = [&](int q, bool qu, std::initializer_list<std::pair<int, int>> ctrl, const std::vector<int> &addr,
                  const std::vector<double> &tab) {
    SvOp op;
    SvGate &g = op.g;
    if (qu) {
      g.mask = bit(L.st0) | bit(L.st1);
      g.v0 = bit(L.st0);   // Q = |st1 st0> = |01>
      g.v1 = bit(L.st1);   // U = |10>
      g.nbits = 2;
      g.pos[0] = std::min(L.st0, L.st1);
      g.pos[1] = std::max(L.st0, L.st1);
    } else {
      g.mask = bit(q);
      g.v0 = 0;
      g.v1 = bit(q);
      g.nbits = 1;
      g.pos[0] = q;
    }
    g.cmask = g.cval = 0;
    for (const auto &cv : ctrl) {
      g.cmask |= bit(cv.first);
      if (cv.second) g.cval |= bit(cv.first);
    }
    g.naddr = (int)addr.size();
    for (int j = 0; j < g.naddr; ++j) g.addr[j] = addr[j];
    op.table_off = K.tables.size();
    K.tables.insert(K.tables.end(), tab.begin(), tab.end());
    K.ops.push_back(op);
  };
  auto ry = [](double th) {
    const double cc = std::cos(0.5 * th), ss = std::sin(0.5 * th);
    return std::vector<double>{cc, -ss, ss, cc};
  };
  auto ry_table = [&](const std::vector<double> &th) {
    std::vector<double> t;
    t.reserve(4 * th.size());
    for (double v : th) {
      const std::vector<double> r = ry(v);
      t.insert(t.end(), r.begin(), r.end());
    }
    return t;
  };
  auto reg = [](int b0, int width) {
    std::vector<int> v;
    for (int j = 0; j < width; ++j) v.push_back(b0 + j);
    return v;
  };
  const std::vector<int> cell = [&] {
    std::vector<int> v = reg(L.x0, L.qx);
    const std::vector<int> y = reg(L.y0, L.qy);
    v.insert(v.end(), y.begin(), y.end());
    return v;
  }();
  const std::vector<int> pair = [&] {   // table index k + nd d
    std::vector<int> v = reg(L.dout0, L.qd);
    const std::vector<int> d = reg(L.din0, L.qd);
    v.insert(v.end(), d.begin(), d.end());
    return v;
  }();
  const std::vector<double> X = {0.0, 1.0, 1.0, 0.0}, Zg = {1.0, 0.0, 0.0, -1.0};
  const double rh = 1.0 / std::sqrt(2.0);
  const std::vector<double> H = {rh, rh, rh, -rh};
  // emission: LCU of I, X, ZX with weights 1/2, 1/4, 1/4 on (em1, em0)
  const double t1 = 2.0 * std::acos(std::sqrt(0.75)), t0 = 2.0 * std::acos(std::sqrt(2.0 / 3.0));
  gate(L.em1, false, {}, {}, ry(t1));
  gate(L.em0, false, {{L.em1, 0}}, {}, ry(t0));
  gate(L.sl, false, {{L.em0, 1}}, {}, X);
  gate(L.sl, false, {{L.em1, 1}}, {}, X);
  gate(L.sl, false, {{L.em1, 1}}, {}, Zg);
  gate(L.em0, false, {{L.em1, 0}}, {}, ry(-t0));
  gate(L.em1, false, {}, {}, ry(-t1));
  // absorption: R_y(2 arccos(a (2 - s) / lambda_max)) per cell on the live sector
  {
    std::vector<double> th(C);
    for (int i = 0; i < C; ++i)
      th[i] = 2.0 * std::acos(std::min(1.0, std::max(-1.0, aabs[i] * (2.0 - surv[i]) / lam_max)));
    gate(L.abs, false, {{L.sl, 0}}, cell, ry_table(th));
  }
  // scattering: selector, PREP_joint, SELECT (d_out ^= d_in, d_out ^= route),
  // RPR, PREP_joint^dagger, selector^dagger
  std::vector<double> th_sel(C);
  for (int i = 0; i < C; ++i) {
    const double s = surv[i];
    th_sel[i] = 2.0 * std::atan(s > 0.0 ? std::sqrt(2.0 * (1.0 - s) / s) : INFINITY);
  }
  gate(L.sel, false, {{L.sl, 0}}, cell, ry_table(th_sel));
  auto prep_level = [&](int lev, bool inverse) {
    const int nb = L.qd - lev;   // sets route bit nb - 1
    std::vector<int> addr = reg(L.din0, L.qd);
    for (int j = 0; j < lev; ++j) addr.push_back(L.route0 + nb + j);
    std::vector<double> th((size_t)nd << lev, 0.0);
    for (int pre = 0; pre < (1 << lev); ++pre)
      for (int d = 0; d < nd; ++d) {
        const int lo = pre << nb;
        double node = 0.0, left = 0.0;
        if (d < n) {
          for (int k = lo; k < lo + (1 << nb); ++k) node += w[k * nd + d];
          for (int k = lo; k < lo + (1 << (nb - 1)); ++k) left += w[k * nd + d];
        }
        const double v = node > 0.0 ? 2.0 * std::acos(std::sqrt(std::min(1.0, left / node))) : 0.0;
        th[(size_t)pre * nd + d] = inverse ? -v : v;
      }
    gate(L.route0 + nb - 1, false, {{L.sl, 0}, {L.sel, 1}}, addr, ry_table(th));
  };
  for (int lev = 0; lev < L.qd; ++lev) prep_level(lev, false);
  for (int j = 0; j < L.qd; ++j) gate(L.dout0 + j, false, {{L.sl, 0}, {L.sel, 1}, {L.din0 + j, 1}}, {}, X);
  for (int j = 0; j < L.qd; ++j) gate(L.dout0 + j, false, {{L.sl, 0}, {L.sel, 1}, {L.route0 + j, 1}}, {}, X);
  auto rot_table = [&](const std::vector<double> &a2) {
    std::vector<double> t;
    for (double v : a2) {
      const double c2 = std::cos(v), s2 = std::sin(v);
      t.insert(t.end(), {c2, s2, -s2, c2});
    }
    return t;
  };
  gate(0, true, {{L.sl, 0}, {L.sel, 1}}, pair, rot_table(sin2));
  gate(L.st0, false, {{L.sl, 0}, {L.sel, 1}}, {}, H);
  {
    std::vector<int> addr = pair;
    addr.push_back(L.st0);
    addr.push_back(L.st1);
    std::vector<double> th(nd * nd * 4);
    for (size_t i = 0; i < th.size(); ++i) th[i] = 2.0 * std::acos(std::min(1.0, std::max(-1.0, 0.5 * lam[i])));
    gate(L.pt, false, {{L.sl, 0}, {L.sel, 1}}, addr, ry_table(th));
  }
  gate(L.st0, false, {{L.sl, 0}, {L.sel, 1}}, {}, H);
  gate(0, true, {{L.sl, 0}, {L.sel, 1}}, pair, rot_table(sout2));
  for (int lev = L.qd - 1; lev >= 0; --lev) prep_level(lev, true);
  for (double &v : th_sel) v = -v;
  gate(L.sel, false, {{L.sl, 0}}, cell, ry_table(th_sel));
  // streaming per axis: R_y(theta(d_out)) on the axis ancilla, the
  // translation by floor(l) + b, R_y(-theta)
  for (int axis = 0; axis < 2; ++axis) {
    const int anc = axis == 0 ? L.ax : L.ay, esc = axis == 0 ? L.ex : L.ey;
    std::vector<double> th(nd, 0.0);
    const int boff = (int)K.bases.size();
    K.bases.resize(K.bases.size() + nd, 0);
    for (int d = 0; d < n; ++d) {
      const double l = axis == 0 ? hp.lx[d] : hp.ly[d];
      const double i0 = std::floor(l), f = l - i0;
      K.bases[boff + d] = (int32_t)i0;
      th[d] = 2.0 * std::asin(std::sqrt(f));
    }
    const std::vector<int> dout = reg(L.dout0, L.qd);
    gate(anc, false, {{L.sl, 0}}, dout, ry_table(th));
    SvOp op;
    op.shift = true;
    op.s.r0 = axis == 0 ? L.x0 : L.y0;
    op.s.qr = axis == 0 ? L.qx : L.qy;
    op.s.ebit = esc;
    op.s.abit = anc;
    op.s.slbit = L.sl;
    op.s.d0 = L.dout0;
    op.s.qd = L.qd;
    op.s.periodic = c->prob.bc[axis == 0 ? 0 : 2] == RT_BC_PERIODIC ? 1 : 0;
    op.base_off = boff;
    K.ops.push_back(op);
    for (double &v : th) v = -v;
    gate(anc, false, {{L.sl, 0}}, dout, ry_table(th));
  }
  return "";
}

// The launches of one step: a translation, a gate alone, or a run of
// consecutive gates on at most max_q target qubits in one pass, where that
// moves fewer statevector bytes (a gate alone moves the pairs whose control
// qubits match: 2^(1 - fixed) of the vector, fixed = its target and control
// qubits; a fused pass moves the states whose shared control qubits match
// once: 2^-shared of it).  With max_q >= 1 the plan also follows the
// statevector's support: the encoded state has every ancilla in |0>, and
// until a gate or a translation first acts on an ancilla each amplitude with
// it at 1 is zero; a launch before then takes the ancilla as a control fixed
// to 0 and skips those amplitudes (a gate maps a pair of zeros to zeros, so
// the nonzero amplitudes get the same products).  Such an amplitude is never
// read at all: the planned step does not zero the vector but writes the
// whole data block (every ancilla 0) when it encodes, and the first launch on
// an ancilla takes its 1 half as zero instead of reading it, then writes both
// halves.
struct SvLaunch {
  int kind = 0;             // 0 translation, 1 gate, 2 fused run
  std::vector<int> ops;     // indices into SvCircuit::ops
  std::vector<int> tq;      // fused: target qubits, ascending
  uint64_t ccmask = 0, ccval = 0;   // fused: control qubits every gate shares, with their value
  int zlocal = 0;           // fused: local states with a never-written target at 1
  int ezero = 0;            // translation: its escape marker never set before
  SvGate g{};               // gate alone: the gate with the untouched ancillas as 0-controls
};

double sv_gate_fraction(const SvGate &g, int nq) {
  int fixed = 0;
  for (int b = 0; b < nq; ++b) fixed += (int)(((g.mask | g.cmask) >> b) & 1);
  return std::ldexp(1.0, 1 - fixed);
}

std::vector<SvLaunch> sv_plan(const SvCircuit &K, int max_q) {
  std::vector<SvLaunch> out;
  std::vector<int> run;
  std::vector<int> tq;
  const int nq = K.L.nq;
  // ancillas not yet acted on (bits ndata .. nq - 1 are the ancillas)
  uint64_t zero = max_q >= 1 ? (((1ull << nq) - 1) & ~((1ull << K.L.ndata) - 1)) : 0;
  uint64_t zero_at_run = zero;
  auto targets = [](const SvGate &g) { return g.mask; };
  auto alone = [&](int i, uint64_t z) {
    SvLaunch l;
    l.kind = 1;
    l.ops = {i};
    l.g = K.ops[i].g;
    l.g.cmask |= z & ~l.g.mask & ~l.g.cmask;   // untouched ancillas: 0-controls
    l.g.zread = l.g.mask & z;                   // a target's 1 half never written yet
    out.push_back(l);
  };
  auto flush = [&]() {
    if (run.empty()) return;
    uint64_t tmask = 0;
    for (int q : tq) tmask |= 1ull << q;
    // each gate alone, with the ancillas untouched before it as 0-controls
    double frac = 0.0;
    {
      uint64_t z = zero_at_run;
      for (int i : run) {
        SvGate g = K.ops[i].g;
        g.cmask |= z & ~g.mask & ~g.cmask;
        frac += sv_gate_fraction(g, nq);
        z &= ~targets(K.ops[i].g);
      }
    }
    // shared controls: the same value in every gate, none of them a target;
    // then the ancillas no gate of the run acts on, fixed to 0
    uint64_t cm = ~0ull;
    for (int i : run) cm &= K.ops[i].g.cmask & ~(K.ops[i].g.cval ^ K.ops[run[0]].g.cval);
    cm &= ~tmask;
    const uint64_t cv = K.ops[run[0]].g.cval & cm;
    const uint64_t zfix = zero_at_run & ~tmask & ~cm;
    const double fused = std::ldexp(1.0, -__builtin_popcountll(cm | zfix));
    if (run.size() >= 2 && frac > fused) {
      SvLaunch l;
      l.kind = 2;
      l.ops = run;
      l.tq = tq;
      std::sort(l.tq.begin(), l.tq.end());
      l.ccmask = cm | zfix;
      l.ccval = cv;
      for (int k = 0; k < (int)l.tq.size(); ++k)
        if ((zero_at_run >> l.tq[k]) & 1) l.zlocal |= 1 << k;
      out.push_back(l);
    } else {
      uint64_t z = zero_at_run;
      for (int i : run) {
        alone(i, z);
        z &= ~targets(K.ops[i].g);
      }
    }
    run.clear();
    tq.clear();
  };
  for (int i = 0; i < (int)K.ops.size(); ++i) {
    const SvOp &op = K.ops[i];
    if (op.shift) {
      flush();
      SvLaunch l;
      l.kind = 0;
      l.ops = {i};
      // zero ancillas: their outputs are written without a read
      l.ccmask = zero & ~(1ull << op.s.ebit) & ~(((1ull << op.s.qr) - 1) << op.s.r0);
      l.ezero = (int)((zero >> op.s.ebit) & 1);
      out.push_back(l);
      zero &= ~(1ull << op.s.ebit);   // the translation marks escapes
      continue;
    }
    std::vector<int> t = tq;
    for (int k = 0; k < op.g.nbits; ++k)
      if (std::find(t.begin(), t.end(), op.g.pos[k]) == t.end()) t.push_back(op.g.pos[k]);
    if (!run.empty() && ((int)t.size() > max_q || (int)run.size() == kSvFuseMaxGates)) {
      flush();
      t.clear();
      for (int k = 0; k < op.g.nbits; ++k) t.push_back(op.g.pos[k]);
    }
    if ((int)t.size() > max_q) {   // max_q 0 (or a pair gate at max_q 1): alone
      flush();
      alone(i, zero);
      zero &= ~targets(op.g);
      continue;
    }
    if (run.empty()) zero_at_run = zero;
    run.push_back(i);
    tq = t;
    zero &= ~targets(op.g);
  }
  flush();
  return out;
}

// Statevector bytes the launches of a plan move: 8 per amplitude read or
// written (amplitudes taken as zero are not read; a translation's reads of
// never-marked sources are not counted, nor are the few that an absorbing
// edge still makes).
double sv_plan_bytes(const SvCircuit &K, const std::vector<SvLaunch> &plan) {
  const int nq = K.L.nq;
  double bytes = 0.0;
  for (const SvLaunch &l : plan) {
    if (l.kind == 1) {
      int fixed = 0;
      for (int b = 0; b < nq; ++b) fixed += (int)(((l.g.mask | l.g.cmask) >> b) & 1);
      const double pairs = std::ldexp(1.0, nq - fixed);
      const int zr = (int)((l.g.zread & l.g.v1) != 0) + (int)((l.g.zread & l.g.v0) != 0);
      bytes += pairs * 8.0 * (2 + 2 - zr);
    } else if (l.kind == 2) {
      uint64_t fixedmask = l.ccmask;
      for (int q : l.tq) fixedmask |= 1ull << q;
      const int m = (int)l.tq.size();
      int reads = 0;
      for (int j = 0; j < (1 << m); ++j) reads += (j & l.zlocal) ? 0 : 1;
      bytes += std::ldexp(1.0, nq - __builtin_popcountll(fixedmask)) * 8.0 * ((1 << m) + reads);
    } else {
      const double read = std::ldexp(1.0, -__builtin_popcountll(l.ccmask)) * (l.ezero ? 0.5 : 1.0);
      bytes += std::ldexp(1.0, nq) * 8.0 * (1.0 + read);
    }
  }
  return bytes;
}

// The fused pass of a planned run; table pointers into the device table region.
SvFuse sv_fuse_of(const SvCircuit &K, const SvLaunch &l, const double *tables) {
  SvFuse f{};
  f.m = (int)l.tq.size();
  f.ngates = (int)l.ops.size();
  for (int k = 0; k < f.m; ++k) f.tq[k] = l.tq[k];
  f.ccmask = l.ccmask;
  f.ccval = l.ccval;
  f.zlocal = l.zlocal;
  auto local = [&](int q) { return (int)(std::find(l.tq.begin(), l.tq.end(), q) - l.tq.begin()); };
  for (int j = 0; j < f.ngates; ++j) {
    const SvOp &op = K.ops[l.ops[j]];
    SvFusedGate &g = f.g[j];
    g.cmask = op.g.cmask;
    g.cval = op.g.cval;
    g.table = tables + op.table_off;
    g.naddr = op.g.naddr;
    for (int q = 0; q < g.naddr; ++q) g.addr[q] = op.g.addr[q];
    if (op.g.nbits == 1) {
      g.code = local(op.g.pos[0]);
    } else {
      int b0 = 0, b1 = 0;
      while (!((op.g.v0 >> b0) & 1)) ++b0;
      while (!((op.g.v1 >> b1) & 1)) ++b1;
      g.code = 3 + 3 * local(b0) + local(b1);
    }
  }
  return f;
}

struct SvWork {
  size_t psi0, psi1, tables, J, partial, norms, bases, total;
};

SvWork sv_work_layout(const SvLayout &L, size_t ntables, size_t nJ, size_t nbases) {
  SvWork W{};
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  W.psi0 = take(sizeof(double) << L.nq);
  W.psi1 = take(sizeof(double) << L.nq);
  W.tables = take(ntables * sizeof(double));
  W.J = take(nJ * sizeof(double));
  W.partial = take((size_t)sv_norm_partials() * sizeof(double));
  W.norms = take(4 * sizeof(double));
  W.bases = take(nbases * sizeof(int32_t));
  W.total = off;
  return W;
}

}  // namespace

extern "C" {

rt_status rt_sv_qubits(const rt_ctx *c, int32_t *nqubits, int32_t *ndata) {
  if (!c || !nqubits) return set_err(RT_EINVAL, "NULL argument");
  SvLayout L;
  const std::string why = sv_check(c, &L);
  if (!why.empty()) return set_err(RT_EUNSUPPORTED, why);
  *nqubits = L.nq;
  if (ndata) *ndata = L.ndata;
  return RT_OK;
}

size_t rt_sv_workspace_bytes(const rt_ctx *c) {
  if (!c) return 0;
  // the tables' sizes do not depend on the medium: compile with a neutral one
  const size_t C = (size_t)c->hp.nx * c->hp.ny;
  std::vector<float> z(C, 0.0f);
  SvCircuit K;
  const std::string why = sv_compile(c, z, z, z, &K);
  if (!why.empty()) {
    set_err(RT_EUNSUPPORTED, why);
    return 0;
  }
  return sv_work_layout(K.L, K.tables.size(), K.J.size(), K.bases.size()).total;
}

rt_status rt_sv_step(rt_ctx *c, void *d_work, size_t work_bytes, const double *d_S_in, double *d_S_out,
                     double *h_psucc) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (!d_work || !d_S_in || !d_S_out) return c->fail(RT_EINVAL, "NULL pointer");
  if (!c->medium_set) return c->fail(RT_ESTATE, "rt_set_medium has not succeeded");
  const HostPlan &hp = c->hp;
  const size_t C = (size_t)hp.nx * hp.ny;
  std::vector<float> tau(C), alb(C), emis(C);
  rt_status st = c->hip(hipMemcpyAsync(tau.data(), c->at<float>(c->L.tau), C * 4, hipMemcpyDeviceToHost, c->stream),
                        "medium");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(alb.data(), c->at<float>(c->L.alb), C * 4, hipMemcpyDeviceToHost, c->stream), "medium");
  if (st == RT_OK)
    st = c->hip(hipMemcpyAsync(emis.data(), c->at<float>(c->L.emis), C * 4, hipMemcpyDeviceToHost, c->stream), "medium");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(c->stream), "medium");
  if (st != RT_OK) return st;
  SvCircuit K;
  const std::string why = sv_compile(c, tau, alb, emis, &K);
  if (!why.empty()) return c->fail(RT_EUNSUPPORTED, why);
  const SvLayout &L = K.L;
  const SvWork W = sv_work_layout(L, K.tables.size(), K.J.size(), K.bases.size());
  if (work_bytes < W.total) return c->fail(RT_ENOMEM, "workspace smaller than rt_sv_workspace_bytes()");
  char *ws = static_cast<char *>(d_work);
  double *psi[2] = {reinterpret_cast<double *>(ws + W.psi0), reinterpret_cast<double *>(ws + W.psi1)};
  double *tables = reinterpret_cast<double *>(ws + W.tables);
  double *J = reinterpret_cast<double *>(ws + W.J);
  double *partial = reinterpret_cast<double *>(ws + W.partial);
  double *norms = reinterpret_cast<double *>(ws + W.norms);   // [0] ||phi_0||^2, [1] p_succ
  int32_t *bases = reinterpret_cast<int32_t *>(ws + W.bases);
  hipStream_t s = c->stream;
  st = c->hip(hipMemcpyAsync(tables, K.tables.data(), K.tables.size() * 8, hipMemcpyHostToDevice, s), "sv tables");
  if (st == RT_OK) st = c->hip(hipMemcpyAsync(J, K.J.data(), K.J.size() * 8, hipMemcpyHostToDevice, s), "sv source");
  if (st == RT_OK && !K.bases.empty())
    st = c->hip(hipMemcpyAsync(bases, K.bases.data(), K.bases.size() * 4, hipMemcpyHostToDevice, s), "sv bases");
  const uint64_t nstates = 1ull << L.nq, nfield = (uint64_t)hp.n * 4 * C;
  // the planned step (fusion on) never reads an amplitude it has not
  // written, so it only encodes the data block; launching every gate over the
  // whole vector needs the vector zeroed
  const bool planned = c->sv_fuse >= 1;
  if (st == RT_OK && !planned) st = c->hip(sv_launch_zero(psi[0], nstates, s), "sv zero");
  if (st == RT_OK) st = c->hip(sv_launch_norm2(d_S_in, nfield, J, nfield, partial, norms, s), "sv norm");
  if (st == RT_OK)
    st = c->hip(planned ? sv_launch_encode_block(psi[0], d_S_in, J, hp.n, L.nd, hp.ny, hp.nx, norms, s)
                        : sv_launch_encode(psi[0], d_S_in, J, hp.n, L.nd, hp.ny, hp.nx, norms, s),
                "sv encode");
  int cur = 0;
  for (const SvLaunch &l : sv_plan(K, c->sv_fuse)) {
    if (st != RT_OK) break;
    if (l.kind == 2) {
      st = c->hip(sv_launch_fused(psi[cur], L.nq, sv_fuse_of(K, l, tables), s), "sv fused gates");
      continue;
    }
    SvOp op = K.ops[l.ops[0]];
    if (op.shift) {
      op.s.base = bases + op.base_off;
      op.s.zmask = l.ccmask;
      op.s.ezero = l.ezero;
      st = c->hip(sv_launch_shift(psi[cur], psi[cur ^ 1], L.nq, op.s, s), "sv shift");
      cur ^= 1;
    } else {
      SvGate g = l.g;
      g.table = tables + op.table_off;
      st = c->hip(sv_launch_gate(psi[cur], L.nq, g, s), "sv gate");
    }
  }
  const uint64_t nblock = 1ull << L.ndata;
  if (st == RT_OK) st = c->hip(sv_launch_norm2(psi[cur], nblock, nullptr, 0, partial, norms + 1, s), "sv p_succ");
  if (st == RT_OK)
    st = c->hip(sv_launch_decode(psi[cur], d_S_out, hp.n, L.nd, hp.ny, hp.nx, 2.0 * K.lam_max, norms, s), "sv decode");
  double hn[2] = {0.0, 0.0};
  if (st == RT_OK) st = c->hip(hipMemcpyAsync(hn, norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "sv norms");
  if (st == RT_OK) st = c->hip(hipStreamSynchronize(s), "sv step");
  if (st == RT_OK && h_psucc) *h_psucc = hn[0] > 0.0 ? hn[1] : 0.0;
  return st;
}

rt_status rt_sv_gate_count(const rt_ctx *c, int32_t *ngates, int32_t *nshifts, double *bytes_per_step) {
  if (!c || !ngates) return set_err(RT_EINVAL, "NULL argument");
  const size_t C = (size_t)c->hp.nx * c->hp.ny;
  std::vector<float> z(C, 0.0f);
  SvCircuit K;
  const std::string why = sv_compile(c, z, z, z, &K);
  if (!why.empty()) return set_err(RT_EUNSUPPORTED, why);
  int g = 0, sh = 0;
  for (const SvOp &op : K.ops) (op.shift ? sh : g) += 1;
  *ngates = g;
  if (nshifts) *nshifts = sh;
  if (bytes_per_step) *bytes_per_step = sv_plan_bytes(K, sv_plan(K, c->sv_fuse));
  return RT_OK;
}

rt_status rt_sv_set_fusion(rt_ctx *c, int32_t max_qubits) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  if (max_qubits < 0 || max_qubits > kSvFuseMaxQ) return c->fail(RT_EINVAL, "max_qubits must lie in 0 .. 3");
  c->sv_fuse = max_qubits;
  return RT_OK;
}

rt_status rt_sv_launch_count(const rt_ctx *c, int32_t *nlaunches) {
  if (!c || !nlaunches) return set_err(RT_EINVAL, "NULL argument");
  const size_t C = (size_t)c->hp.nx * c->hp.ny;
  std::vector<float> z(C, 0.0f);
  SvCircuit K;
  const std::string why = sv_compile(c, z, z, z, &K);
  if (!why.empty()) return set_err(RT_EUNSUPPORTED, why);
  *nlaunches = (int32_t)sv_plan(K, c->sv_fuse).size();
  return RT_OK;
}

// ---------------------------------------------------------------- spectral batch

}  // extern "C"

// The batch's tuning table, from timing every admissible setting on the
// 64-channel spectral workload (bench.py --batch-autotune prints the
// measurement; bf16, forward steps):
//  * cache budget of the temporal blocking: the working set of a channel
//    group.  All channels stepping together take 4.37 ms per step (4.4 GB
//    of state stream through HBM every step); groups of up to 64-192 MiB
//    3.63-3.67 ms (a group's states stay in the 256 MiB last-level cache
//    from one step to the next); one channel per group 3.62 ms.  128 MiB
//    keeps the small channels batched at the same speed.
//  * block waves per class (waves per tile W): 8-wave blocks for every
//    class (W = 2: 3.72 ms against 3.73 for 2-wave blocks; W = 4: 3.67
//    against 3.72).
constexpr size_t kBatchCacheBudget = 128u << 20;

int batch_block_waves(int prec, int W) {
  (void)prec;
  (void)W;
  return kBatchWaves;
}

struct rt_batch {
  int nchan = 0;
  std::vector<rt_ctx *> ch;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  // device descriptor tables: forward run, forward recompute in the adjoint, adjoint
  BatchChan *d_run = nullptr, *d_rec = nullptr, *d_adj = nullptr;
  std::vector<BatchChan> h_run, h_rec, h_adj;   // per channel, channel order
  // A class is the channels with the same waves per tile W (= Rpad / 32);
  // its launches use blocks of bw waves (bw / W tiles side by side).
  struct Class {
    int W = 0, bw = 0, lds = 0, count = 0;
    int lds_dich = 0;   // LDS of a run with dichroic absorption (its adjoint keeps a fourth per-cell sum)
  };
  std::vector<Class> classes;   // increasing W
  // Temporal blocking: the channels are split into groups whose working set
  // fits the cache budget, and a run or adjoint completes every step of one
  // group before the next (the channels are independent, so the order does
  // not change any result); within a group a step is one persistent launch
  // per class, over one (group, class) run of the device tables.
  struct Run {
    int first = 0, count = 0, cls = 0;
    int64_t nitems = 0;
    int ext = kExtNone;   // kExtMix / kExtDich: a channel of the run has a phase mixture / dichroic absorption
  };
  struct Group {
    std::vector<Run> runs;
    std::vector<int> chans;
  };
  struct Plan {
    std::vector<Group> groups;
    std::vector<int> order;   // channel of each table entry
  } plan_run, plan_adj;
  size_t cache_budget = kBatchCacheBudget;
  std::vector<BatchChan> t_run, t_rec, t_adj;    // staged tables, table order
  int prec = 0;
  int cu_count = 0;   // compute units of the device (each launch sizes its own grid)
  bool graph_mode = false;
  hipStream_t cap = nullptr;   // private stream graphs are recorded on (the caller's may be the null stream)
  struct Graph {
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  } g_run, g_adj;
  std::string err;

  rt_status fail(rt_status s, const std::string &m) {
    err = m;
    g_last_error = m;
    return s;
  }
  rt_status hip(hipError_t e, const char *where) {
    if (e == hipSuccess) return RT_OK;
    return fail(RT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
  }
  static void drop(Graph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = Graph{};
  }
  ~rt_batch() {
    drop(g_run);
    drop(g_adj);
    if (cap) (void)hipStreamDestroy(cap);
    for (rt_ctx *c : ch) delete c;
  }
  // A channel with dichroic absorption needs its class's dichroic LDS.
  rt_status check_dichroic() {
    for (int i = 0; i < nchan; ++i) {
      if (!ch[i]->dichroic) continue;
      for (const Class &k : classes)
        if (k.W == ch[i]->geo.Rpad / 32 && k.lds_dich == 0)
          return fail(RT_EUNSUPPORTED, "channel " + std::to_string(i) +
                                           ": the dichroic adjoint's per-cell sums do not fit the LDS at this block size");
    }
    return RT_OK;
  }
  // The step arguments of every channel as its context now stands (a phase
  // mixture set or removed since the batch was made changes them; the
  // medium lives in the context's workspace and needs no refresh).
  void refresh_args() {
    for (int i = 0; i < nchan; ++i) {
      h_run[i].a = ch[i]->args(false);
      h_rec[i].a = h_run[i].a;
      h_adj[i].a = ch[i]->args(true);
      h_run[i].a.strip = h_rec[i].a.strip = h_adj[i].a.strip = 0;   // tiles in row order
      // (a group's states stay in the last-level cache from step to step)
      h_run[i].a.nt_out = h_rec[i].a.nt_out = h_adj[i].a.nt_out = 0;
    }
  }
  rt_status upload(BatchChan *d, const std::vector<BatchChan> &h, const Plan &pl) {
    std::vector<BatchChan> &t = d == d_run ? t_run : (d == d_rec ? t_rec : t_adj);
    t.resize(h.size());
    for (size_t k = 0; k < pl.order.size(); ++k) t[k] = h[pl.order[k]];
    return hip(hipMemcpyAsync(d, t.data(), t.size() * sizeof(BatchChan), hipMemcpyHostToDevice, stream),
               "batch descriptors");
  }
  rt_status step(const BatchChan *d, const Group &gr, bool adjoint, bool gather, bool ckpt, const BatchSel &sel) {
    if (gr.chans.size() == 1) {
      // a group of one channel runs that channel's single-problem kernel (the
      // same tile arithmetic; without the batch kernel's channel bookkeeping)
      const int i = gr.chans[0];
      rt_ctx *c = ch[i];
      const std::vector<BatchChan> &tb = d == d_run ? h_run : (d == d_rec ? h_rec : h_adj);
      auto bufp = [&](int id, int slot) -> float * {
        return id < 0 ? nullptr : tb[i].buf[id] + (int64_t)slot * tb[i].state_elems;
      };
      StepArgs a = c->args(adjoint);
      a.in = bufp(sel.in, sel.in_slot);
      a.out = bufp(sel.out, sel.out_slot);
      a.s_out = ckpt ? bufp(sel.sout, sel.sout_slot) : nullptr;
      a.lam_next = bufp(sel.lam, sel.lam_slot);
      return hip(adjoint ? launch_adjoint_mfma(a, prec, gather, stream, c->cu_count)
                         : launch_step_mfma(a, prec, gather, stream, c->cu_count),
                 "batch step");
    }
    for (const Run &r : gr.runs) {
      const Class &k = classes[r.cls];
      rt_status st = hip(launch_batch_step(d + r.first, r.count, r.nitems, prec, k.bw, adjoint, gather, ckpt,
                                           r.ext, sel, r.ext == kExtDich ? k.lds_dich : k.lds, cu_count, stream),
                         "batch step");
      if (st != RT_OK) return st;
    }
    return RT_OK;
  }
  // LDS and kernel attributes of every class for its block size.
  rt_status configure() {
    for (Class &k : classes) {
      const int Rpad = 32 * k.W;
      const size_t lf = batch_lds_bytes(Rpad, prec, false, k.bw), la = batch_lds_bytes(Rpad, prec, true, k.bw);
      const size_t ld = batch_lds_bytes(Rpad, prec, true, k.bw, true);
      if (lf == (size_t)-1 || la == (size_t)-1 || ld == (size_t)-1)
        return fail(RT_EINVAL, "block waves do not fit the channel class");
      const size_t lds = std::max(lf, la), lds_dich = std::max(lf, ld);
      if (lds > 160 * 1024) return fail(RT_EUNSUPPORTED, "batch does not fit the fused kernel's LDS budget");
      k.lds = (int)lds;
      k.lds_dich = lds_dich <= 160 * 1024 ? (int)lds_dich : 0;   // 0: no dichroic channel in this class
      int per_cu = 0;
      rt_status st = hip(prepare_batch(prec, k.bw, std::max(k.lds, k.lds_dich), &per_cu), "prepare batch kernels");
      if (st != RT_OK) return st;
    }
    return RT_OK;
  }
  // Groups of channels (in channel order) whose working sets, `states`
  // states each, add up to at most the cache budget (a larger channel is a
  // group of its own; budget 0: one group), their (group, class) runs of the
  // tables, and the work items of every channel in `tables`.
  void make_plan(Plan &pl, double states, std::initializer_list<std::vector<BatchChan> *> tables) {
    pl.groups.clear();
    pl.order.clear();
    std::vector<std::vector<int>> members;
    double used = 0.0;
    for (int i = 0; i < nchan; ++i) {
      const double bytes = states * (double)state_elems(ch[i]) * sizeof(float);
      if (members.empty() || (cache_budget > 0 && used + bytes > (double)cache_budget)) {
        members.emplace_back();
        used = 0.0;
      }
      members.back().push_back(i);
      used += bytes;
    }
    for (const std::vector<int> &m : members) {
      Group gr;
      gr.chans = m;
      for (int c = 0; c < (int)classes.size(); ++c) {
        // the channels with dichroic absorption run apart from the others
        // (a launch carries one extension: the mixture tile takes channels
        // without a mixture exactly, the dichroic tile those without factors)
        for (const bool dich : {false, true}) {
          Run r;
          r.cls = c;
          r.first = (int)pl.order.size();
          r.ext = dich ? kExtDich : kExtNone;
          const int W = classes[c].W, per = classes[c].bw / W;
          int64_t item = 0;
          for (int i : m) {
            if (ch[i]->geo.Rpad / 32 != W || ch[i]->dichroic != dich) continue;
            pl.order.push_back(i);
            if (ch[i]->mixture) r.ext = kExtMix;
            for (std::vector<BatchChan> *tb : tables) {
              (*tb)[i].groups = per;
              (*tb)[i].item0 = item;
            }
            item += (h_run[i].ntiles + per - 1) / per;
          }
          r.count = (int)pl.order.size() - r.first;
          r.nitems = item;
          if (r.count > 0) gr.runs.push_back(r);
        }
      }
      pl.groups.push_back(gr);
    }
  }
  // Records body() into a graph unless the cached one has the same key, then
  // launches it on the caller's stream.  Recording happens on a private
  // stream (body() enqueues on `stream`, which points there meanwhile).
  template <typename F>
  rt_status graphed(Graph &g, const std::vector<uintptr_t> &key, F body) {
    if (!(g.exec && g.key == key)) {
      drop(g);
      if (!cap) {
        rt_status sc = hip(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        if (sc != RT_OK) return sc;
      }
      rt_status st = hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
      if (st != RT_OK) return st;
      hipStream_t user = stream;
      stream = cap;
      rt_status sb = body();
      stream = user;
      hipGraph_t graph = nullptr;
      st = hip(hipStreamEndCapture(cap, &graph), "end capture");
      if (sb != RT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return sb;
      }
      if (st != RT_OK) return st;
      hipGraphExec_t exec = nullptr;
      st = hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate graph");
      if (st != RT_OK) {
        (void)hipGraphDestroy(graph);
        return st;
      }
      g.graph = graph;
      g.exec = exec;
      g.key = key;
    }
    return hip(hipGraphLaunch(g.exec, stream), "launch graph");
  }
};

namespace {

BatchSel sel_of(int in, int in_slot, int out, int out_slot, int sout = kBufNone, int sout_slot = 0,
                int lam = kBufNone, int lam_slot = 0) {
  BatchSel b;
  b.in = in;
  b.in_slot = in_slot;
  b.out = out;
  b.out_slot = out_slot;
  b.sout = sout;
  b.sout_slot = sout_slot;
  b.lam = lam;
  b.lam_slot = lam_slot;
  return b;
}

// Work-queue offsets of the channels inside the workspace.
struct BatchPlan {
  std::vector<size_t> off, bytes;
  size_t table_off = 0, table_bytes = 0, total = 0;
};

rt_status batch_plan(const rt_problem *probs, int32_t nchan, BatchPlan *bp, std::string *msg) {
  if (!probs || nchan < 1) {
    *msg = "need at least one channel";
    return RT_EINVAL;
  }
  bp->table_off = 0;
  bp->table_bytes = align256(3 * (size_t)nchan * sizeof(BatchChan));
  size_t off = bp->table_bytes;
  for (int i = 0; i < nchan; ++i) {
    const rt_problem &p = probs[i];
    rt_status st = rt_validate(&p);
    if (st != RT_OK) {
      *msg = "channel " + std::to_string(i) + ": " + g_last_error;
      return st;
    }
    if (p.plane == RT_PLANE_3D) {
      *msg = "3-D lattices cannot be batched";
      return RT_EUNSUPPORTED;
    }
    if (p.flags & RT_PLAIN) {
      *msg = "RT_PLAIN channels cannot be batched";
      return RT_EUNSUPPORTED;
    }
    if (p.precision != probs[0].precision || p.flags != probs[0].flags) {
      *msg = "channel " + std::to_string(i) + ": precision and flags must match channel 0";
      return RT_EINVAL;
    }
    const int n = p.n_zen * p.n_az;
    const int Rpad = (4 * n + 31) / 32 * 32;
    if (Rpad / 32 > kBatchWaves || kBatchWaves % (Rpad / 32) != 0) {
      *msg = "channel " + std::to_string(i) + ": batching needs 4n padded to 32, 64, 128 or 256";
      return RT_EUNSUPPORTED;
    }
    const size_t b = align256(rt_workspace_bytes(&p));
    bp->off.push_back(off);
    bp->bytes.push_back(b);
    off += b;
  }
  bp->total = off;
  return RT_OK;
}

// Block waves per class of the batched step (waves per tile W = Rpad / 32):
// the tuning table, from timing every admissible block size on the 64-channel
// spectral workload (bench.py --batch-autotune prints the measurement).  One
// tile group per block for W >= 2: wider blocks keep their tile groups in
// step through the block's barriers, where independent blocks overlap.
rt_status batch_set_err(rt_batch *b, rt_status s, const std::string &m) {
  if (b) return b->fail(s, m);
  g_last_error = m;
  return s;
}

}  // namespace

extern "C" {

const char *rt_batch_last_error(const rt_batch *b) { return b ? b->err.c_str() : g_last_error.c_str(); }

size_t rt_batch_workspace_bytes(const rt_problem *probs, int32_t nchan) {
  BatchPlan bp;
  std::string msg;
  if (batch_plan(probs, nchan, &bp, &msg) != RT_OK) return 0;
  return bp.total;
}

rt_status rt_batch_init(const rt_problem *probs, int32_t nchan, void *d_ws, size_t ws_bytes, void *stream,
                        rt_batch **out) {
  if (!out) return set_err(RT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_ws) return set_err(RT_EINVAL, "workspace is NULL");
  BatchPlan bp;
  std::string msg;
  rt_status st = batch_plan(probs, nchan, &bp, &msg);
  if (st != RT_OK) return set_err(st, msg);
  if (ws_bytes < bp.total) return set_err(RT_ENOMEM, "workspace smaller than rt_batch_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return set_err(RT_EINVAL, "workspace not 256-byte aligned");
  rt_batch *b = new rt_batch;
  b->nchan = nchan;
  b->stream = static_cast<hipStream_t>(stream);
  b->ws = static_cast<char *>(d_ws);
  b->prec = probs[0].precision;
  for (int i = 0; i < nchan; ++i) {
    rt_ctx *c = nullptr;
    st = rt_init(&probs[i], b->ws + bp.off[i], bp.bytes[i], stream, &c);
    if (st != RT_OK) {
      const std::string m = "channel " + std::to_string(i) + ": " + g_last_error;
      delete b;
      return set_err(st, m);
    }
    b->ch.push_back(c);
  }
  b->d_run = reinterpret_cast<BatchChan *>(b->ws + bp.table_off);
  b->d_rec = b->d_run + nchan;
  b->d_adj = b->d_rec + nchan;
  for (int i = 0; i < nchan; ++i) {
    rt_ctx *c = b->ch[i];
    BatchChan f{};
    f.a = c->args(false);
    f.a.strip = 0;   // the batched kernel numbers its tiles in row order
    f.a.nt_out = 0;  // and keeps a group's states in the last-level cache
    f.buf[kBufYa] = c->at<float>(c->L.Ya);
    f.buf[kBufYb] = c->at<float>(c->L.Yb);
    f.buf[kBufLa] = c->at<float>(c->L.La);
    f.buf[kBufLb] = c->at<float>(c->L.Lb);
    f.state_elems = (int64_t)state_elems(c);
    f.ntiles = (c->geo.C + 31) / 32;
    BatchChan a = f;
    a.a = c->args(true);
    a.a.strip = 0;
    a.a.nt_out = 0;
    b->h_run.push_back(f);
    b->h_rec.push_back(f);
    b->h_adj.push_back(a);
  }
  // classes by waves per tile, in increasing W
  for (int W = 1; W <= kBatchWaves; W *= 2) {
    rt_batch::Class k;
    k.W = W;
    k.bw = batch_block_waves(b->prec, W);
    for (int i = 0; i < nchan; ++i) k.count += b->ch[i]->geo.Rpad / 32 == W;
    if (k.count > 0) b->classes.push_back(k);
  }
  b->cu_count = b->ch[0]->cu_count;
  st = b->configure();
  if (st == RT_OK) st = b->hip(hipStreamSynchronize(b->stream), "batch init");
  if (st != RT_OK) {
    const std::string m = b->err;
    delete b;
    return set_err(st, m);
  }
  *out = b;
  return RT_OK;
}

rt_status rt_batch_channel(rt_batch *b, int32_t ch, rt_ctx **out) {
  if (!b || !out) return batch_set_err(b, RT_EINVAL, "NULL batch or out");
  if (ch < 0 || ch >= b->nchan) return b->fail(RT_EINVAL, "channel index out of range");
  *out = b->ch[ch];
  return RT_OK;
}

rt_status rt_batch_run(rt_batch *b, float *const *h_states, int32_t nsteps, float *const *h_ckpt,
                       int32_t ckpt_every) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  if (!h_states) return b->fail(RT_EINVAL, "NULL state array");
  if (nsteps < 0) return b->fail(RT_EINVAL, "nsteps < 0");
  if (h_ckpt && ckpt_every < 1) return b->fail(RT_EINVAL, "ckpt_every < 1");
  for (int i = 0; i < b->nchan; ++i) {
    if (!h_states[i] || (h_ckpt && !h_ckpt[i])) return b->fail(RT_EINVAL, "NULL state or checkpoint pointer");
    if (!b->ch[i]->medium_set) return b->fail(RT_ESTATE, "rt_set_medium has not succeeded on every channel");
  }
  if (nsteps == 0) return RT_OK;
  if (b->check_dichroic() != RT_OK) return RT_EUNSUPPORTED;
  b->refresh_args();
  // a step reads one post-collision state and writes the other
  b->make_plan(b->plan_run, 2.0, {&b->h_run});
  auto body = [&]() -> rt_status {
    rt_status st = RT_OK;
    for (const rt_batch::Group &gr : b->plan_run.groups) {
      if (h_ckpt)
        for (int i : gr.chans)
          if (st == RT_OK)
            st = b->hip(hipMemcpyAsync(h_ckpt[i], h_states[i], state_elems(b->ch[i]) * sizeof(float),
                                       hipMemcpyDeviceToDevice, b->stream), "ckpt");
      if (st == RT_OK) st = b->step(b->d_run, gr, false, false, false, sel_of(kBufS, 0, kBufYa, 0));
      for (int t = 1; t < nsteps && st == RT_OK; ++t) {
        const int yin = (t - 1) & 1 ? kBufYb : kBufYa, yout = t & 1 ? kBufYb : kBufYa;
        const bool ck = h_ckpt && t % ckpt_every == 0;
        st = b->step(b->d_run, gr, false, true, ck,
                     sel_of(yin, 0, yout, 0, ck ? kBufCkpt : kBufNone, ck ? t / ckpt_every : 0));
      }
      const int ylast = (nsteps - 1) & 1 ? kBufYb : kBufYa;
      for (int i : gr.chans)
        if (st == RT_OK)
          st = b->hip(launch_stream(b->ch[i]->args(false), b->h_run[i].buf[ylast], h_states[i], b->stream),
                      "stream");
    }
    return st;
  };
  for (int i = 0; i < b->nchan; ++i) {
    b->h_run[i].buf[kBufS] = h_states[i];
    b->h_run[i].buf[kBufCkpt] = h_ckpt ? h_ckpt[i] : nullptr;
  }
  if (!b->graph_mode) {
    rt_status st = b->upload(b->d_run, b->h_run, b->plan_run);
    return st == RT_OK ? body() : st;
  }
  std::vector<uintptr_t> key = {1, (uintptr_t)nsteps, (uintptr_t)ckpt_every, (uintptr_t)(h_ckpt != nullptr)};
  for (int i = 0; i < b->nchan; ++i) {
    key.push_back(reinterpret_cast<uintptr_t>(h_states[i]));
    key.push_back(reinterpret_cast<uintptr_t>(h_ckpt ? h_ckpt[i] : nullptr));
    // the kernels and tables the channel needs
    key.push_back((uintptr_t)(b->ch[i]->mixture ? b->ch[i]->nmix : 0) | (b->ch[i]->dichroic ? 1u << 16 : 0u));
  }
  if (!(b->g_run.exec && b->g_run.key == key)) {
    rt_status st = b->upload(b->d_run, b->h_run, b->plan_run);
    if (st != RT_OK) return st;
  }
  return b->graphed(b->g_run, key, body);
}

rt_status rt_batch_adjoint(rt_batch *b, int32_t nsteps, float *const *h_ckpt, int32_t ckpt_every,
                           float *const *h_seg, float *const *h_lambdaT, float *const *h_g_tau,
                           float *const *h_g_albedo, float *const *h_g_emis) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  if (!h_ckpt || !h_lambdaT || !h_g_tau || !h_g_albedo || !h_g_emis)
    return b->fail(RT_EINVAL, "NULL pointer array");
  if (nsteps < 1 || ckpt_every < 1) return b->fail(RT_EINVAL, "nsteps and ckpt_every must be >= 1");
  if (ckpt_every > 1 && !h_seg) return b->fail(RT_EINVAL, "segment buffers are NULL");
  for (int i = 0; i < b->nchan; ++i) {
    if (!h_ckpt[i] || !h_lambdaT[i] || !h_g_tau[i] || !h_g_albedo[i] || !h_g_emis[i] ||
        (ckpt_every > 1 && !h_seg[i]))
      return b->fail(RT_EINVAL, "NULL per-channel pointer");
    if (!b->ch[i]->medium_set) return b->fail(RT_ESTATE, "rt_set_medium has not succeeded on every channel");
  }
  if (b->check_dichroic() != RT_OK) return RT_EUNSUPPORTED;
  b->refresh_args();
  // a reverse step reads lambda_{t+1}, the segment state and writes lambda_t;
  // the segment recompute writes ckpt_every - 1 states
  b->make_plan(b->plan_adj, 3.0 + ckpt_every, {&b->h_rec, &b->h_adj});
  auto body = [&]() -> rt_status {
    rt_status st = RT_OK;
    for (const rt_batch::Group &gr : b->plan_adj.groups) {
      for (int i : gr.chans) {
        rt_ctx *c = b->ch[i];
        if (st == RT_OK) st = b->hip(launch_fill_f64(c->at<double>(c->L.gacc), 4 * c->geo.C, 0.0, b->stream), "fill");
      }
      int lam = kBufLamT;
      int flip = 0;
      const int nseg = (nsteps + ckpt_every - 1) / ckpt_every;
      for (int k = nseg - 1; k >= 0 && st == RT_OK; --k) {
        const int t0 = k * ckpt_every;
        const int t1 = std::min(nsteps, t0 + ckpt_every);
        if (t1 - t0 >= 2) {
          st = b->step(b->d_rec, gr, false, false, false, sel_of(kBufCkpt, k, kBufSeg, 0));
          for (int t = t0 + 1; t <= t1 - 2 && st == RT_OK; ++t)
            st = b->step(b->d_rec, gr, false, true, false, sel_of(kBufSeg, t - 1 - t0, kBufSeg, t - t0));
        }
        for (int t = t1 - 1; t >= t0 && st == RT_OK; --t) {
          const bool gather = t > t0;
          const int out = flip ? kBufLb : kBufLa;
          st = b->step(b->d_adj, gr, true, gather, false,
                       sel_of(gather ? kBufSeg : kBufCkpt, gather ? t - 1 - t0 : k, out, 0, kBufNone, 0, lam, 0));
          lam = out;
          flip ^= 1;
        }
      }
      for (int i : gr.chans) {
        rt_ctx *c = b->ch[i];
        if (st == RT_OK)
          st = b->hip(launch_gradchain(c->geo.C, c->at<float>(c->L.tau), c->at<float>(c->L.alb), c->prob.flags,
                                       c->at<double>(c->L.gacc), h_g_tau[i], h_g_albedo[i], h_g_emis[i], b->stream,
                                       c->dichroic ? c->at<float>(c->L.dich_eta) : nullptr),
                      "gradchain");
      }
    }
    return st;
  };
  for (int i = 0; i < b->nchan; ++i)
    for (std::vector<BatchChan> *tb : {&b->h_rec, &b->h_adj}) {
      (*tb)[i].buf[kBufCkpt] = h_ckpt[i];
      (*tb)[i].buf[kBufSeg] = h_seg ? h_seg[i] : nullptr;
      (*tb)[i].buf[kBufLamT] = h_lambdaT[i];
    }
  auto upload_both = [&]() -> rt_status {
    rt_status st = b->upload(b->d_rec, b->h_rec, b->plan_adj);
    return st == RT_OK ? b->upload(b->d_adj, b->h_adj, b->plan_adj) : st;
  };
  if (!b->graph_mode) {
    rt_status st = upload_both();
    return st == RT_OK ? body() : st;
  }
  std::vector<uintptr_t> key = {2, (uintptr_t)nsteps, (uintptr_t)ckpt_every};
  for (int i = 0; i < b->nchan; ++i) {
    for (const void *ptr : {(const void *)h_ckpt[i], (const void *)(h_seg ? h_seg[i] : nullptr),
                            (const void *)h_lambdaT[i], (const void *)h_g_tau[i], (const void *)h_g_albedo[i],
                            (const void *)h_g_emis[i]})
      key.push_back(reinterpret_cast<uintptr_t>(ptr));
    key.push_back((uintptr_t)(b->ch[i]->mixture ? b->ch[i]->nmix : 0) | (b->ch[i]->dichroic ? 1u << 16 : 0u));
  }
  if (!(b->g_adj.exec && b->g_adj.key == key)) {
    rt_status st = upload_both();
    if (st != RT_OK) return st;
  }
  return b->graphed(b->g_adj, key, body);
}

rt_status rt_batch_num_classes(const rt_batch *b, int32_t *h_count) {
  if (!b || !h_count) return set_err(RT_EINVAL, "NULL batch or count");
  *h_count = (int32_t)b->classes.size();
  return RT_OK;
}

rt_status rt_batch_class(const rt_batch *b, int32_t k, int32_t *h_waves_per_tile, int32_t *h_block_waves,
                         int32_t *h_nchan) {
  if (!b || !h_waves_per_tile || !h_block_waves || !h_nchan) return set_err(RT_EINVAL, "NULL pointer");
  if (k < 0 || k >= (int32_t)b->classes.size()) return set_err(RT_EINVAL, "class index out of range");
  *h_waves_per_tile = b->classes[k].W;
  *h_block_waves = b->classes[k].bw;
  *h_nchan = b->classes[k].count;
  return RT_OK;
}

rt_status rt_batch_set_cache_budget(rt_batch *b, size_t bytes) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  b->cache_budget = bytes;
  rt_batch::drop(b->g_run);   // recorded graphs hold the old grouping
  rt_batch::drop(b->g_adj);
  return RT_OK;
}

rt_status rt_batch_set_tuning(rt_batch *b, int32_t waves_per_tile, int32_t block_waves) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  rt_batch::Class *cls = nullptr;
  for (rt_batch::Class &k : b->classes)
    if (k.W == waves_per_tile) cls = &k;
  if (!cls) return b->fail(RT_EINVAL, "no channel class with that many waves per tile");
  if (block_waves < waves_per_tile || block_waves > kBatchWaves || block_waves % waves_per_tile != 0 ||
      (block_waves & (block_waves - 1)) != 0)
    return b->fail(RT_EINVAL, "block waves must be a power-of-two multiple of the waves per tile, at most 8");
  const int old = cls->bw;
  cls->bw = block_waves;
  rt_status st = b->configure();
  if (st != RT_OK) {
    cls->bw = old;
    (void)b->configure();
    return st;
  }
  // recorded graphs hold the old launches and work-item counts
  rt_batch::drop(b->g_run);
  rt_batch::drop(b->g_adj);
  return RT_OK;
}

rt_status rt_batch_set_graph(rt_batch *b, int32_t enabled) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  if (enabled != 0 && enabled != 1) return b->fail(RT_EINVAL, "enabled must be 0 or 1");
  b->graph_mode = enabled == 1;
  if (!b->graph_mode) {
    rt_batch::drop(b->g_run);
    rt_batch::drop(b->g_adj);
  }
  return RT_OK;
}

rt_status rt_batch_synchronize(rt_batch *b) {
  if (!b) return set_err(RT_EINVAL, "batch is NULL");
  return b->hip(hipStreamSynchronize(b->stream), "synchronize");
}

rt_status rt_batch_destroy(rt_batch *b) {
  delete b;
  return RT_OK;
}

rt_status rt_synchronize(rt_ctx *c) {
  if (!c) return set_err(RT_EINVAL, "context is NULL");
  return c->hip(hipStreamSynchronize(c->stream), "synchronize");
}

rt_status rt_destroy(rt_ctx *c) {
  delete c;
  return RT_OK;
}

}  // extern "C"
