// Host setup of the polarized LBM solver: problem validation, direction grid,
// lattice displacements, the collision matrix and its packing into MFMA lane
// fragments.  Float64 throughout; no HIP calls.
//
// The collision matrix is built here from the field picture of dipole
// scattering: a field E_in in the meridian frame (e_theta, e_phi) of the
// incoming direction scatters into (1 - k_out k_out^T) E_in, whose components
// in the outgoing meridian frame form the real 2x2 Jones matrix
// A_ij = e_i(out) . e_j(in).  Its Mueller matrix equals the rotation-phase-
// rotation product R(psi_out) P(theta) R(psi_in) of Eq. 13 with the Rayleigh
// matrix of Eq. 16 (a different construction of the same operator).  Each 4x4
// block is the Eq. 17 weight times the Mueller matrix normalised to its I->I
// element, so the I->I blocks of a column sum to one (Sec. 2.1.1).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "rt_internal.h"

namespace rtl {

namespace {

constexpr double kPi = 3.14159265358979323846;

double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// A displacement component within 1e-12 of an integer is that integer: the
// cosine of a 90 degree azimuth evaluates to 6e-17, which would otherwise
// give an axis-aligned direction a vanishing cross-axis displacement (a tap of
// weight 6e-17 in Eq. 34 and a place among the directions leaving through
// that axis's edge).
double snap_integer(double l) {
  const double r = std::nearbyint(l);
  return std::fabs(l - r) < 1e-12 ? r : l;
}

// Scalar phase function normalised over 4 pi (Rayleigh: 3/(16 pi)(1 + c^2)).
double phase_fn(int kind, double c, double g, double mix) {
  const double pr = 3.0 / (16.0 * kPi) * (1.0 + c * c);
  if (kind == RT_PHASE_RAYLEIGH) return pr;
  const double den = 1.0 + g * g - 2.0 * g * c;
  const double phg = (1.0 - g * g) / (4.0 * kPi * den * std::sqrt(den));
  if (kind == RT_PHASE_HG) return phg;
  return mix * pr + (1.0 - mix) * phg;
}

// The six elements (a1, a2, a3, a4, b1, b2) of a tabulated scattering matrix
// at cos(theta) = c: linear in theta (degrees) between the rows
// (theta_deg, a1, a2, a3, a4, b1, b2) of `tab`, whose angles rise from 0 to 180.
void table_elements(const double *tab, int rows, double c, double *f) {
  // acos loses half the digits next to +-1: cosines within 1e-12 of +-1 take
  // the forward / backward rows
  const double th = c >= 1.0 - 1e-12 ? 0.0 : (c <= -1.0 + 1e-12 ? 180.0 : std::acos(c) * (180.0 / kPi));
  int lo = 0, hi = rows - 1;   // tab[lo][0] <= th <= tab[hi][0]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (tab[7 * mid] <= th) lo = mid; else hi = mid;
  }
  const double t0 = tab[7 * lo], t1 = tab[7 * hi];
  const double u = (th - t0) / (t1 - t0);
  for (int j = 0; j < 6; ++j) {
    const double v0 = tab[7 * lo + 1 + j], v1 = tab[7 * hi + 1 + j];
    f[j] = u <= 0.0 ? v0 : (u >= 1.0 ? v1 : v0 + u * (v1 - v0));
  }
}

// Mueller matrix (row-major 4x4) of a real Jones matrix a = [[a11,a12],[a21,a22]]
// acting on (E_theta, E_phi):  I = |E1|^2+|E2|^2, Q = |E1|^2-|E2|^2,
// U = 2 Re(E1 E2*), V proportional to Im(E1 E2*).
void jones_to_mueller(double a11, double a12, double a21, double a22, double *Z) {
  const double s11 = a11 * a11, s12 = a12 * a12, s21 = a21 * a21, s22 = a22 * a22;
  Z[0] = 0.5 * (s11 + s12 + s21 + s22);
  Z[1] = 0.5 * (s11 - s12 + s21 - s22);
  Z[2] = a11 * a12 + a21 * a22;
  Z[3] = 0.0;
  Z[4] = 0.5 * (s11 + s12 - s21 - s22);
  Z[5] = 0.5 * (s11 - s12 - s21 + s22);
  Z[6] = a11 * a12 - a21 * a22;
  Z[7] = 0.0;
  Z[8] = a11 * a21 + a12 * a22;
  Z[9] = a11 * a21 - a12 * a22;
  Z[10] = a11 * a22 + a12 * a21;
  Z[11] = 0.0;
  Z[12] = 0.0;
  Z[13] = 0.0;
  Z[14] = 0.0;
  Z[15] = a11 * a22 - a12 * a21;
}

// Pair matrix of a tabulated scattering matrix, Eq. 13 with F in place of the
// Rayleigh matrix: the field components in the incoming meridian axes
// (e_theta, e_phi) are projected onto the scattering-plane axes (e_par, n),
// F acts there, and the result is projected onto the outgoing meridian axes.
// Both projections are real rotations; their Mueller matrices are the frame
// rotations of Eq. 21.  n = k_in x k_out normalised (e_phi of the incoming
// direction where k_out = +-k_in), e_par = n x k.
void table_pair(const HostPlan &hp, const double *tab, int rows, int dout, int di, double *Z) {
  const double *ki = &hp.kvec[3 * di], *ko = &hp.kvec[3 * dout];
  const double *eti = &hp.eth[3 * di], *epi = &hp.eph[3 * di];
  const double *eto = &hp.eth[3 * dout], *epo = &hp.eph[3 * dout];
  double nv[3] = {ki[1] * ko[2] - ki[2] * ko[1], ki[2] * ko[0] - ki[0] * ko[2], ki[0] * ko[1] - ki[1] * ko[0]};
  const double nn = std::sqrt(dot3(nv, nv));
  if (nn < 1e-12) {
    for (int j = 0; j < 3; ++j) nv[j] = epi[j];
  } else {
    for (int j = 0; j < 3; ++j) nv[j] /= nn;
  }
  auto cross = [](const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  double pin[3], pout[3];
  cross(nv, ki, pin);
  cross(nv, ko, pout);
  double Rin[16], Rout[16];
  jones_to_mueller(dot3(pin, eti), dot3(pin, epi), dot3(nv, eti), dot3(nv, epi), Rin);
  jones_to_mueller(dot3(eto, pout), dot3(eto, nv), dot3(epo, pout), dot3(epo, nv), Rout);
  double f[6];
  table_elements(tab, rows, dot3(ko, ki), f);
  const double F[16] = {f[0], f[4], 0.0, 0.0, f[4], f[1], 0.0, 0.0, 0.0, 0.0, f[2], f[5], 0.0, 0.0, -f[5], f[3]};
  double T[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += F[4 * r + k] * Rin[4 * k + c];
      T[4 * r + c] = acc;
    }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += Rout[4 * r + k] * T[4 * k + c];
      Z[4 * r + c] = acc;
    }
}

std::string fmt(const char *what, double v) {
  std::ostringstream o;
  o << what << " (" << v << ")";
  return o.str();
}

}  // namespace

int gemm_row(int n, int d, int s) {
  (void)n;
  return 4 * d + s;
}

rt_status build_plan(const rt_problem *p, HostPlan *hp, std::string *msg) {
  if (!p) { *msg = "problem is NULL"; return RT_EINVAL; }
  if (p->nx < 1 || p->ny < 1) { *msg = "nx and ny must be >= 1"; return RT_EINVAL; }
  if (p->plane < 0 || p->plane > 3) { *msg = "plane out of range"; return RT_EINVAL; }
  const bool three_d = p->plane == RT_PLANE_3D;
  if (three_d && p->nz < 1) { *msg = "nz must be >= 1 for RT_PLANE_3D"; return RT_EINVAL; }
  if (!three_d && p->nz > 1) { *msg = "nz > 1 needs RT_PLANE_3D"; return RT_EINVAL; }
  const int nlay = three_d ? p->nz : 1;   // layers of the lattice
  if (p->n_zen < 1 || p->n_az < 1) { *msg = "n_zen and n_az must be >= 1"; return RT_EINVAL; }
  const long long n = (long long)p->n_zen * p->n_az;
  if (n > kMaxDirs) { *msg = "n_zen * n_az must be <= 256"; return RT_EINVAL; }
  const long long cells = (long long)p->nx * p->ny * nlay;
  if (cells * 4 * n > (1LL << 40)) { *msg = "state larger than 2^40 elements"; return RT_EINVAL; }
  if (cells >= (1LL << 31)) { *msg = "nx * ny (* nz) must be < 2^31"; return RT_EINVAL; }
  if (p->zen_rule < 0 || p->zen_rule > 2) { *msg = "zen_rule out of range"; return RT_EINVAL; }
  if (p->mix_max < 0 || p->mix_max > RT_MIX_MAX) { *msg = "mix_max must lie in 0 .. RT_MIX_MAX"; return RT_EINVAL; }
  if (p->zen_rule == RT_ZEN_EXPLICIT && !p->zen_deg) { *msg = "zen_deg is NULL for RT_ZEN_EXPLICIT"; return RT_EINVAL; }
  if (!std::isfinite(p->az_offset_deg)) { *msg = "az_offset_deg not finite"; return RT_EINVAL; }
  if (three_d) {
    for (int e = 0; e < 2; ++e)
      if (p->bc_z[e] < 0 || p->bc_z[e] > 2) { *msg = "bc_z value out of range"; return RT_EINVAL; }
    if ((p->bc_z[0] == RT_BC_PERIODIC) != (p->bc_z[1] == RT_BC_PERIODIC)) {
      *msg = "both z faces must be periodic or neither"; return RT_EINVAL;
    }
  }
  if (p->plane != RT_PLANE_XY_D2Q9 && !(std::isfinite(p->courant) && p->courant > 0)) {
    *msg = fmt("courant must be finite and > 0", p->courant); return RT_EINVAL;
  }
  for (int e = 0; e < 4; ++e)
    if (p->bc[e] < 0 || p->bc[e] > 2) { *msg = "bc value out of range"; return RT_EINVAL; }
  if ((p->bc[0] == RT_BC_PERIODIC) != (p->bc[1] == RT_BC_PERIODIC) ||
      (p->bc[2] == RT_BC_PERIODIC) != (p->bc[3] == RT_BC_PERIODIC)) {
    *msg = "both edges of an axis must be periodic or neither"; return RT_EINVAL;
  }
  if (p->phase < 0 || p->phase > 3) { *msg = "phase out of range"; return RT_EINVAL; }
  if ((p->phase == RT_PHASE_HG || p->phase == RT_PHASE_MIX) && !(std::isfinite(p->g) && std::fabs(p->g) < 1.0)) {
    *msg = fmt("HG asymmetry must satisfy |g| < 1", p->g); return RT_EINVAL;
  }
  if (p->phase == RT_PHASE_MIX && !(p->mix_ray >= 0.0 && p->mix_ray <= 1.0)) {
    *msg = fmt("mix_ray must lie in [0, 1]", p->mix_ray); return RT_EINVAL;
  }
  if (p->phase == RT_PHASE_TABLE) {
    const int rows = p->n_table;
    const double *t = p->table;
    if (!t) { *msg = "table is NULL for RT_PHASE_TABLE"; return RT_EINVAL; }
    if (rows < 2 || rows > 65536) { *msg = fmt("n_table must lie in [2, 65536]", rows); return RT_EINVAL; }
    for (int r = 0; r < rows; ++r) {
      for (int j = 0; j < 7; ++j)
        if (!std::isfinite(t[7 * r + j])) { *msg = fmt("table entry not finite in row", r); return RT_EINVAL; }
      if (!(t[7 * r + 1] > 0.0)) { *msg = fmt("table a1 must be > 0; row", r); return RT_EINVAL; }
      if (r > 0 && !(t[7 * r] > t[7 * (r - 1)])) {
        *msg = fmt("table angles must increase strictly; row", r); return RT_EINVAL;
      }
    }
    if (t[0] != 0.0 || t[7 * (rows - 1)] != 180.0) {
      *msg = "table angles must run from exactly 0 to exactly 180 degrees"; return RT_EINVAL;
    }
    // forward / backward rows must not depend on the (undefined) scattering plane
    const double *f = t, *b = t + 7 * (rows - 1);
    const double tf = 1e-6 * f[1], tb = 1e-6 * b[1];
    if (std::fabs(f[5]) > tf || std::fabs(f[6]) > tf || std::fabs(f[3] - f[2]) > tf || std::fabs(b[5]) > tb ||
        std::fabs(b[6]) > tb || std::fabs(b[3] + b[2]) > tb) {
      *msg = "table rows at 0 and 180 degrees depend on the scattering plane (need b1 = b2 = 0, "
             "a3 = a2 forward, a3 = -a2 backward)";
      return RT_EINVAL;
    }
  }
  if (!(std::isfinite(p->dt) && p->dt >= 0)) { *msg = fmt("dt must be finite and >= 0", p->dt); return RT_EINVAL; }
  const uint32_t known = RT_ABS_TAYLOR | RT_SCAT_EXP | RT_FUSED_TAYLOR | RT_RENORM_IROW | RT_SCALAR | RT_PLAIN;
  if (p->flags & ~known) { *msg = "unknown flag bits"; return RT_EINVAL; }
  if ((p->flags & RT_FUSED_TAYLOR) && (p->flags & (RT_ABS_TAYLOR | RT_SCAT_EXP))) {
    *msg = "RT_FUSED_TAYLOR excludes RT_ABS_TAYLOR and RT_SCAT_EXP"; return RT_EINVAL;
  }
  if (p->precision < 0 || p->precision > 3) { *msg = "precision out of range"; return RT_EINVAL; }
  // explicit direction set
  if (p->dir_xyz) {
    for (long long d = 0; d < n; ++d) {
      const double *k = p->dir_xyz + 3 * d;
      if (!(std::isfinite(k[0]) && std::isfinite(k[1]) && std::isfinite(k[2]))) {
        *msg = fmt("dir_xyz not finite for direction", (double)d); return RT_EINVAL;
      }
      if (std::fabs(std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]) - 1.0) > 1e-9) {
        *msg = fmt("dir_xyz is not a unit vector for direction", (double)d); return RT_EINVAL;
      }
      if (std::hypot(k[0], k[1]) < 1e-9) {
        *msg = fmt("dir_xyz along the polar axis (no meridian plane) for direction", (double)d); return RT_EINVAL;
      }
    }
  }
  if (p->dir_domega) {
    for (long long d = 0; d < n; ++d)
      if (!(std::isfinite(p->dir_domega[d]) && p->dir_domega[d] > 0.0)) {
        *msg = fmt("dir_domega must be finite and > 0; direction", (double)d); return RT_EINVAL;
      }
  }
  if (p->shift) {
    const int dim = three_d ? 3 : 2;
    for (long long i = 0; i < n * dim; ++i) {
      if (!std::isfinite(p->shift[i])) { *msg = "shift not finite"; return RT_EINVAL; }
      if (std::fabs(p->shift[i]) > 1.0 + 1e-12) {
        *msg = fmt("shift: displacement per step exceeds one cell", p->shift[i]); return RT_ERANGE;
      }
    }
  }
  if ((p->flags & RT_PLAIN) && p->precision != RT_FP32) {
    *msg = "RT_PLAIN is a float32 path"; return RT_EUNSUPPORTED;
  }

  hp->nx = p->nx;
  hp->ny = p->ny * nlay;
  hp->nz = nlay;
  hp->ny_lattice = p->ny;
  hp->n = (int)n;
  hp->R = 4 * hp->n;
  hp->Rpad = (hp->R + kTileRows - 1) / kTileRows * kTileRows;
  const int nz = p->n_zen, na = p->n_az;

  // Zenith and azimuth nodes, d = i_zen * n_az + j_az.
  std::vector<double> zen(nz);
  for (int i = 0; i < nz; ++i) {
    if (p->zen_rule == RT_ZEN_EQUAL_AREA) {
      zen[i] = std::acos(1.0 - (2.0 * i + 1.0) / nz);
    } else if (p->zen_rule == RT_ZEN_UNIFORM_THETA) {
      zen[i] = (i + 1.0) * kPi / (nz + 1.0);
    } else {
      const double z = p->zen_deg[i];
      if (!(std::isfinite(z) && z > 0.0 && z < 180.0)) {
        *msg = fmt("explicit zenith must lie in (0, 180) degrees", z); return RT_EINVAL;
      }
      zen[i] = z * kPi / 180.0;
    }
  }
  hp->theta.resize(n);
  hp->phi.resize(n);
  hp->domega.assign(n, 4.0 * kPi / n);
  if (p->dir_domega) hp->domega.assign(p->dir_domega, p->dir_domega + n);
  hp->kvec.resize(3 * n);
  hp->eth.resize(3 * n);
  hp->eph.resize(3 * n);
  hp->lx.resize(n);
  hp->ly.resize(n);
  hp->lz.assign(n, 0.0);
  hp->outmask.assign(n, 0);
  for (int i = 0; i < nz; ++i) {
    for (int j = 0; j < na; ++j) {
      const int d = i * na + j;
      double *k = &hp->kvec[3 * d], *et = &hp->eth[3 * d], *ep = &hp->eph[3 * d];
      if (p->dir_xyz) {
        std::memcpy(k, p->dir_xyz + 3 * d, 3 * sizeof(double));
      } else {
        const double th = zen[i];
        const double ph = (p->az_offset_deg + 360.0 * j / na) * kPi / 180.0;
        k[0] = std::sin(th) * std::cos(ph); k[1] = std::sin(th) * std::sin(ph); k[2] = std::cos(th);
      }
      // the meridian frame from k, the same for a grid direction and an
      // explicit one (e_phi along increasing azimuth, e_theta = e_phi x k)
      const double st = std::hypot(k[0], k[1]), ct = k[2];
      const double cp = k[0] / st, sp = k[1] / st;
      hp->theta[d] = std::atan2(st, ct);
      hp->phi[d] = std::atan2(k[1], k[0]);
      et[0] = ct * cp; et[1] = ct * sp; et[2] = -st;
      ep[0] = -sp; ep[1] = cp; ep[2] = 0.0;
      double l0, l1;
      if (p->plane == RT_PLANE_3D) {
        l0 = p->courant * k[0]; l1 = p->courant * k[1];
        const double l2 = p->courant * k[2];
        if (std::fabs(l2) > 1.0 + 1e-12) { *msg = fmt("displacement per step exceeds one cell", l2); return RT_ERANGE; }
        hp->lz[d] = std::max(-1.0, std::min(1.0, snap_integer(l2)));
      } else if (p->plane == RT_PLANE_XY) {
        l0 = p->courant * k[0]; l1 = p->courant * k[1];
      } else if (p->plane == RT_PLANE_XZ) {
        l0 = p->courant * k[0]; l1 = p->courant * k[2];
      } else {
        const double c[2] = {cp, sp};
        double l[2];
        for (int a = 0; a < 2; ++a) {
          if (std::fabs(std::fabs(c[a]) - 0.5) < 1e-6) {
            *msg = "azimuth ambiguous for D2Q9 velocities (component near 1/2)"; return RT_EINVAL;
          }
          l[a] = c[a] > 0.5 ? 1.0 : (c[a] < -0.5 ? -1.0 : 0.0);
        }
        l0 = l[0]; l1 = l[1];
      }
      if (p->shift) {
        const int dim = p->plane == RT_PLANE_3D ? 3 : 2;
        l0 = p->shift[dim * d];
        l1 = p->shift[dim * d + 1];
        if (dim == 3) hp->lz[d] = std::max(-1.0, std::min(1.0, snap_integer(p->shift[dim * d + 2])));
      }
      if (std::fabs(l0) > 1.0 + 1e-12 || std::fabs(l1) > 1.0 + 1e-12) {
        *msg = fmt("displacement per step exceeds one cell", std::max(std::fabs(l0), std::fabs(l1)));
        return RT_ERANGE;
      }
      hp->lx[d] = std::max(-1.0, std::min(1.0, snap_integer(l0)));
      hp->ly[d] = std::max(-1.0, std::min(1.0, snap_integer(l1)));
      int m = 0;
      if (hp->lx[d] < 0) m |= 1;
      if (hp->lx[d] > 0) m |= 2;
      if (hp->ly[d] < 0) m |= 4;
      if (hp->ly[d] > 0) m |= 8;
      if (hp->lz[d] < 0) m |= 16;   // 3-D: leaves through z- / z+
      if (hp->lz[d] > 0) m |= 32;
      hp->outmask[d] = m;
    }
  }

  // Eq. 17 weights, column-normalised over outgoing directions.
  const int R = hp->R;
  std::vector<double> w((size_t)n * n);
  for (int di = 0; di < n; ++di) {
    double tot = 0.0;
    for (int dout = 0; dout < n; ++dout) {
      double c = dot3(&hp->kvec[3 * dout], &hp->kvec[3 * di]);
      c = std::max(-1.0, std::min(1.0, c));
      double v;
      if (p->phase == RT_PHASE_TABLE) {
        double f[6];
        table_elements(p->table, p->n_table, c, f);
        v = f[0] * hp->domega[dout];
      } else {
        v = phase_fn(p->phase, c, p->g, p->mix_ray) * hp->domega[dout];
      }
      w[(size_t)dout * n + di] = v;
      tot += v;
    }
    for (int dout = 0; dout < n; ++dout) w[(size_t)dout * n + di] /= tot;
  }

  hp->M.assign((size_t)R * R, 0.0);
  const bool scalar = (p->flags & RT_SCALAR) != 0;
  for (int dout = 0; dout < n; ++dout) {
    for (int di = 0; di < n; ++di) {
      const double wt = w[(size_t)dout * n + di];
      double Z[16];
      if (scalar) {
        std::memset(Z, 0, sizeof(Z));
        Z[0] = 1.0;
      } else if (p->phase == RT_PHASE_TABLE) {
        table_pair(*hp, p->table, p->n_table, dout, di, Z);
        const double z11 = Z[0];
        for (int q = 0; q < 16; ++q) Z[q] /= z11;
      } else {
        const double *eto = &hp->eth[3 * dout], *epo = &hp->eph[3 * dout];
        const double *eti = &hp->eth[3 * di], *epi = &hp->eph[3 * di];
        jones_to_mueller(dot3(eto, eti), dot3(eto, epi), dot3(epo, eti), dot3(epo, epi), Z);
        const double z11 = Z[0];
        for (int q = 0; q < 16; ++q) Z[q] /= z11;
      }
      for (int so = 0; so < 4; ++so)
        for (int si = 0; si < 4; ++si)
          hp->M[(size_t)(4 * dout + so) * R + 4 * di + si] = wt * Z[4 * so + si];
    }
  }
  if ((p->flags & RT_RENORM_IROW) && !scalar) {
    for (int di = 0; di < n; ++di) {
      for (int j = 1; j <= 2; ++j) {
        double tot = 0.0;
        for (int dout = 0; dout < n; ++dout) tot += hp->M[(size_t)(4 * dout) * R + 4 * di + j];
        for (int dout = 0; dout < n; ++dout)
          hp->M[(size_t)(4 * dout) * R + 4 * di + j] -= w[(size_t)dout * n + di] * tot;
      }
    }
  }
  return RT_OK;
}

std::vector<double> gemm_order(const HostPlan &hp) {
  const int n = hp.n, R = hp.R, Rp = hp.Rpad;
  std::vector<double> G((size_t)Rp * Rp, 0.0);
  for (int dout = 0; dout < n; ++dout)
    for (int so = 0; so < 4; ++so)
      for (int di = 0; di < n; ++di)
        for (int si = 0; si < 4; ++si)
          G[(size_t)gemm_row(n, dout, so) * Rp + gemm_row(n, di, si)] =
              hp.M[(size_t)(4 * dout + so) * R + 4 * di + si];
  return G;
}

namespace {

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint16_t to_f16(double v) {
  _Float16 h = (_Float16)(float)v;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

}  // namespace

void pack_fragments(const HostPlan &hp, bool transpose, FragKind kind, double scale, bool lo,
                    std::vector<TileRange> *tiles, std::vector<uint8_t> *bytes) {
  const int Rp = hp.Rpad;
  const std::vector<double> G = gemm_order(hp);
  auto A = [&](int r, int k) -> double {
    return scale * (transpose ? G[(size_t)k * Rp + r] : G[(size_t)r * Rp + k]);
  };
  const int kstep = (kind == FRAG_F32) ? 8 : 16;
  const int ntiles = Rp / kTileRows;
  tiles->assign(ntiles, TileRange{0, 0, 0, 0});
  bytes->clear();
  int rec = 0;
  for (int t = 0; t < ntiles; ++t) {
    int kmin = Rp, kmax = -1;
    for (int r = t * kTileRows; r < (t + 1) * kTileRows; ++r)
      for (int k = 0; k < Rp; ++k)
        if (A(r, k) != 0.0) { kmin = std::min(kmin, k); kmax = std::max(kmax, k); }
    TileRange tr{0, 0, rec, 0};
    if (kmax >= 0) {
      tr.klo = kmin / kstep * kstep;
      tr.khi = std::min(Rp, (kmax / kstep + 1) * kstep);
    }
    for (int kb = tr.klo; kb < tr.khi; kb += kstep) {
      for (int lane = 0; lane < 64; ++lane) {
        const int r = t * kTileRows + lane % 32;
        const int g = lane / 32;
        uint8_t buf[16];
        if (kind == FRAG_F32) {
          float v[4];
          for (int j = 0; j < 4; ++j) {
            const int k = kb + 4 * g + j;
            v[j] = k < Rp ? (float)A(r, k) : 0.0f;
          }
          std::memcpy(buf, v, 16);
        } else {
          uint16_t v[8];
          for (int j = 0; j < 8; ++j) {
            const int k = kb + 8 * g + j;
            const double a = k < Rp ? A(r, k) : 0.0;
            if (kind == FRAG_BF16) {
              const uint16_t hi = to_bf16((float)a);
              v[j] = lo ? to_bf16((float)(a - (double)from_bf16(hi))) : hi;
            } else {
              v[j] = to_f16(a);
            }
          }
          std::memcpy(buf, v, 16);
        }
        bytes->insert(bytes->end(), buf, buf + 16);
        ++rec;
      }
    }
    (*tiles)[t] = tr;
  }
  bytes->insert(bytes->end(), 64 * 16, uint8_t(0));
  for (TileRange &tr : *tiles) tr.zero_off = rec;
}

}  // namespace rtl
