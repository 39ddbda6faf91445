// Host side of libibmlbm: configuration checks, workspace carving, marker
// geometry, launch order of the time step, and read-back.  See ibmlbm.h for
// the contract of every entry point.
#include "ibmlbm.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "divmul.h"
#include "internal.h"
#include "marker_args.h"
#include "kinematics.h"

using namespace ibmk;

namespace {

thread_local std::string g_err;

struct Region {
  size_t off = 0, bytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct LatticeLayout {
  int es = 4;        // bytes per stored value
  int px = 0;
  long long ps = 0;      // population stride (elements)
  size_t total = 0;      // elements of the slabs of one state buffer
  size_t goff = 0;       // byte offset of the ghost records in a state buffer
  size_t N = 0;
  int nxc = 0, nblocks = 0;
  Region fA, fB, mass_part, diag, argtab;
  size_t state_end = 0;  // bytes of the two states
  size_t end = 0;
};

// Launch arguments of a window of kFactorWindow steps, on the device: the
// collide arguments of every slot, then the marker arguments of every slot.
constexpr size_t kArgSlotBytes = sizeof(CollideArgs) + sizeof(MarkerArgs);

struct WingGeom {
  int np = 0;
  double ds = 0.0;                 // perimeter / np
  std::vector<double> ref;         // np x 2, relative to the pivot
  double rmax = 0.0;
  int side = 0;                    // pitch of the per-layer node-box images
  int max_cells = 0;               // largest node box over the motion (cells, with margin)
};

constexpr int kPwStride = 14;      // doubles per perimeter record (markers.hip)

struct MarkerLayout {
  Region ref, G, Minv, pw, sup, T, X, U, B, rhoB, duB, fpart, hist;
  std::vector<Region> band, corr;
  size_t end = 0;
  int m_total = 0, layers = 0, perims = 0;
  int minv_step = 0, pw_step = 0, sup_step = 0;
};

}  // namespace

struct ibmlbm_s {
  ibmlbm_config cfg{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // base of every region other than the two lattice states: the workspace
  // itself, or this device's static scratch for ibmlbm_create_noalloc
  char* sb = nullptr;
  size_t sb_bytes = 0;
  bool noalloc = false;
  LatticeLayout L;
  Geo geo{};
  Phys phys{};
  bool cur_is_A = true;
  bool initialized = false;
  long long step = 0;
  // markers
  int nw = 0;
  ibmlbm_wing wings[kMaxWings]{};
  WingDev wd[kMaxWings]{};
  std::vector<WingGeom> geom;
  MarkerLayout M;
  bool markers_valid = false;       // marker outputs of a completed step exist
  long long win_t0 = -1;            // window of precomputed factors and launch arguments
  std::vector<CollideArgs> wca;     // host copies of the window's arguments
  std::vector<MarkerArgs> wma;
  void* pin = nullptr;              // pinned staging of the window upload
  hipEvent_t pin_ev = nullptr;      // completes when the last upload has been read
  bool pin_pending = false;
  // timing
  bool timing = false;
  int timing_every = 1;             // bracket one step in this many
  std::vector<hipEvent_t> ev;       // pairs: start, stop
  std::vector<int> ev_kind;         // 0 = collide, 1 = markers
  size_t ev_used = 0;
  std::vector<double> ev_cells;      // cells updated by each timed collide launch
  double acc_collide_ms = 0.0, acc_marker_ms = 0.0, acc_collide_cells = 0.0;
  long long acc_collide_n = 0;
  std::string err;
};

namespace {

int fail(ibmlbm_t h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  g_err = buf;
  return code;
}

#define HIP_TRY(h, expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((h), IBMLBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

template <class T>
T* at(ibmlbm_t h, const Region& r) {
  return reinterpret_cast<T*>(h->sb + r.off);
}

void* cur_state(ibmlbm_t h) { return h->ws + (h->cur_is_A ? h->L.fA.off : h->L.fB.off); }
void* next_state(ibmlbm_t h) { return h->ws + (h->cur_is_A ? h->L.fB.off : h->L.fA.off); }

int validate_config(const ibmlbm_config* c, std::string& why) {
  char b[256];
  if (!c) { why = "null config"; return IBMLBM_EINVAL; }
  if (c->nx < 4 || c->ny < 4 || c->nz < 1) { why = "nx, ny must be >= 4 and nz >= 1"; return IBMLBM_EINVAL; }
  // nz = 1 with a periodic span is the 2D scheme: D3Q19 on one periodic
  // layer reduces exactly to D2Q9 (summing the populations that share
  // (c_x, c_y) gives the D2Q9 weights, equilibrium, forcing and streaming)
  if (c->nz < 4 && c->bc[4] != IBMLBM_BC_PERIODIC) { why = "nz < 4 needs a periodic z axis"; return IBMLBM_EINVAL; }
  if ((long long)c->nx * c->ny * c->nz > (1LL << 34)) { why = "box too large"; return IBMLBM_EINVAL; }
  // the kernels index lattice rows (y, z) with 32-bit integers and address a
  // row's 19 population rows with 32-bit byte offsets
  if ((long long)c->ny * c->nz >= (1LL << 31)) { why = "ny * nz must be < 2^31"; return IBMLBM_EINVAL; }
  if (c->nx >= (1 << 24)) { why = "nx must be < 2^24"; return IBMLBM_EINVAL; }
  for (int f = 0; f < 6; ++f) {
    if (c->bc[f] < 0 || c->bc[f] > 5) { snprintf(b, sizeof b, "bc[%d] unknown", f); why = b; return IBMLBM_EINVAL; }
    if (f >= 2 && c->bc[f] >= IBMLBM_BC_VELOCITY) {
      why = "VELOCITY/PRESSURE faces are supported on x faces only";
      return IBMLBM_EINVAL;
    }
  }
  for (int a = 0; a < 3; ++a)
    if ((c->bc[2 * a] == IBMLBM_BC_PERIODIC) != (c->bc[2 * a + 1] == IBMLBM_BC_PERIODIC)) {
      snprintf(b, sizeof b, "axis %d: PERIODIC must be set on both faces", a);
      why = b;
      return IBMLBM_EINVAL;
    }
  if (!(c->tau > 0.5) || !std::isfinite(c->tau)) { why = "tau must be finite and > 0.5"; return IBMLBM_EINVAL; }
  if (c->storage < 0 || c->storage > 2) { why = "unknown storage"; return IBMLBM_EINVAL; }
  if (c->check_interval < 0) { why = "check_interval must be >= 0"; return IBMLBM_EINVAL; }
  if (c->history_steps < 1) { why = "history_steps must be >= 1"; return IBMLBM_EINVAL; }
  if (!(c->rho_out > 0.0)) { why = "rho_out must be > 0"; return IBMLBM_EINVAL; }
  if (!(c->u_ref > 0.0) || !(c->area_ref > 0.0)) { why = "u_ref and area_ref must be > 0"; return IBMLBM_EINVAL; }
  return IBMLBM_OK;
}

// split: the two states alone from offset 0 of the caller's buffer, the
// other regions from offset 0 of a separate scratch (ibmlbm_create_noalloc);
// otherwise everything follows on in one workspace.
LatticeLayout lattice_layout(const ibmlbm_config* c, bool split = false) {
  LatticeLayout L;
  L.es = c->storage == IBMLBM_FP32 ? 4 : 2;
  const int line = 128 / L.es;
  L.px = ((c->nx + 2 + line - 1) / line) * line;
  L.ps = L.px;
  L.total = ((size_t)c->ny * c->nz + 1) * kQ * (size_t)L.px;
  L.N = (size_t)c->nx * c->ny * c->nz;
  L.nxc = (c->nx + kBlockX - 1) / kBlockX;
  L.nblocks = L.nxc * ((c->ny * c->nz + kBlockRows - 1) / kBlockRows);
  size_t o = 0;
  auto take = [&](Region& r, size_t bytes) { r.off = o; r.bytes = bytes; o = align256(o + bytes); };
  L.goff = align256(L.total * L.es);
  const size_t state = L.goff + 2 * (size_t)c->ny * c->nz * 32;
  take(L.fA, state);
  take(L.fB, state);
  L.state_end = o;
  if (split) o = 0;
  take(L.mass_part, (size_t)L.nblocks * sizeof(double));
  take(L.diag, 64);
  take(L.argtab, (size_t)kFactorWindow * kArgSlotBytes);
  L.end = o;
  return L;
}

// ----------------------------------------------------------- host geometry --

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
}

struct Arc {
  double a, b;
  std::vector<double> gx, gw;
  int panels = 512;
  std::vector<double> cum;   // arc length at the start of each panel
  Arc(double a_, double b_) : a(a_), b(b_) {
    gauss_legendre(16, gx, gw);
    const double h = 2.0 * M_PI / panels;
    cum.assign(panels + 1, 0.0);
    for (int k = 0; k < panels; ++k) cum[k + 1] = cum[k] + piece(k * h, (k + 1) * h);
  }
  double speed(double t) const { return std::hypot(a * std::sin(t), b * std::cos(t)); }
  // Gauss-Legendre integral of the speed over [lo, hi]
  double piece(double lo, double hi) const {
    const double c = 0.5 * (lo + hi), r = 0.5 * (hi - lo);
    double acc = 0.0;
    for (size_t j = 0; j < gx.size(); ++j) acc += gw[j] * speed(c + r * gx[j]);
    return r * acc;
  }
  // arc length from 0 to phi (phi in [0, 2 pi]) by composite Gauss-Legendre:
  // whole panels from the table, then the part of the last panel
  double length(double phi) const {
    const double h = 2.0 * M_PI / panels;
    int full = (int)std::floor(phi / h);
    if (full >= panels) return cum[panels];
    if (full < 0) full = 0;
    return cum[full] + (phi > full * h ? piece(full * h, phi) : 0.0);
  }
};

// Equal-arc-length markers on the ellipse of one foil; the first at the
// trailing edge (local (a, 0)), counter-clockwise; coordinates relative to
// the pivot on the chord (pivot_frac 0 = LE at (-a, 0), 1 = TE).
int wing_geometry(const ibmlbm_wing& w, WingGeom& g, std::string& why) {
  if (!(w.chord > 0.0) || !(w.thickness > 0.0) || w.thickness > w.chord || !(w.ds > 0.0)) {
    why = "foil needs chord > 0, 0 < thickness <= chord and ds > 0";
    return IBMLBM_EINVAL;
  }
  const double a = 0.5 * w.chord, b = 0.5 * w.thickness;
  Arc arc(a, b);
  const double P = arc.length(2.0 * M_PI);
  const int n = std::max(3, (int)std::lround(P / w.ds));
  if (n > kMaxPerim) {
    why = "too many perimeter markers (max 128): reduce chord or raise ds";
    return IBMLBM_EINVAL;
  }
  g.np = n;
  g.ds = P / n;
  g.ref.assign(2 * n, 0.0);
  const double xp = -a + 2.0 * a * w.pivot_frac;
  g.rmax = 0.0;
  for (int j = 0; j < n; ++j) {
    const double target = j * g.ds;
    double phi = 2.0 * M_PI * target / P;
    for (int it = 0; it < 60; ++it) {
      const double d = (arc.length(phi) - target) / arc.speed(phi);
      phi -= d;
      if (std::fabs(d) < 1e-15) break;
    }
    const double rx = a * std::cos(phi) - xp, ry = b * std::sin(phi);
    g.ref[2 * j] = rx;
    g.ref[2 * j + 1] = ry;
    g.rmax = std::max(g.rmax, std::hypot(rx, ry));
  }
  return IBMLBM_OK;
}

double delta_h(double r) {
  r = std::fabs(r);
  return r <= 2.0 ? 0.25 * (1.0 + std::cos(0.5 * M_PI * r)) : 0.0;
}

void pose_h(const ibmlbm_wing& w, double t, double& th, double& hx, double& hy) {
  double al = w.alpha_mean;
  if (w.alpha_shape == IBMLBM_ALPHA_SIN) {
    al = w.alpha_mean + w.alpha_amp * std::sin(2.0 * M_PI * t / w.period_steps + w.phase);
  } else if (w.alpha_shape == IBMLBM_ALPHA_ABS_SIN) {
    const double psi = t / w.period_steps + w.phase / (2.0 * M_PI);
    const double h = psi - std::floor(2.0 * psi) / 2.0;
    al = w.alpha_mean + w.alpha_amp * std::sin(2.0 * M_PI * h);
  }
  th = w.theta0 + w.sense * al;
  hx = w.hinge[0];
  hy = w.hinge[1];
  if (w.trans_amp != 0.0) {
    const double A = w.trans_amp * std::cos(2.0 * M_PI * t / w.period_steps + w.phase);
    hx += A * std::cos(w.trans_angle);
    hy += A * std::sin(w.trans_angle);
  }
}

void perimeter_xy(const ibmlbm_wing& w, const WingGeom& g, double t, std::vector<double>& xy) {
  double th, hx, hy;
  pose_h(w, t, th, hx, hy);
  const double c = std::cos(th), s = std::sin(th);
  xy.resize(2 * g.np);
  for (int p = 0; p < g.np; ++p) {
    const double px = g.ref[2 * p], py = g.ref[2 * p + 1];
    xy[2 * p] = hx + (c * px - s * py);
    xy[2 * p + 1] = hy + (s * px + c * py);
  }
}

// Node box of one foil at time t: every support node floor(X)-1 .. floor(X)+2
// of its markers, with one spare cell on each side against rounding
// differences between host and device trigonometry; clipped to the box.
void node_box(const ibmlbm_wing& w, const WingGeom& g, double t, const ibmlbm_config& c,
              WingDev& d) {
  std::vector<double> xy;
  perimeter_xy(w, g, t, xy);
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int p = 0; p < g.np; ++p) {
    x0 = std::min(x0, xy[2 * p]);
    x1 = std::max(x1, xy[2 * p]);
    y0 = std::min(y0, xy[2 * p + 1]);
    y1 = std::max(y1, xy[2 * p + 1]);
  }
  const int bx0 = std::max(0, (int)std::floor(x0) - 2);
  const int bx1 = std::min(c.nx - 1, (int)std::floor(x1) + 3);
  const int by0 = std::max(0, (int)std::floor(y0) - 2);
  const int by1 = std::min(c.ny - 1, (int)std::floor(y1) + 3);
  d.x0 = bx0;
  d.y0 = by0;
  d.bw = std::min(bx1 - bx0 + 1, g.side);
  d.bh = std::min(by1 - by0 + 1, g.side);
}

// Bound on the number of support nodes of a foil at time t in its node box
// d: the marker kernels list the nodes floor(X) - 1 .. floor(X) + 2 of every
// marker from positions they compute themselves; taking both floors of
// X -/+ 1e-9 here gives a set that contains theirs.
int support_bound(const ibmlbm_wing& w, const WingGeom& g, double t, const WingDev& d) {
  std::vector<double> xy;
  perimeter_xy(w, g, t, xy);
  std::vector<unsigned char> hit((size_t)d.bw * d.bh, 0);
  int cnt = 0;
  for (int p = 0; p < g.np; ++p) {
    const int xa = std::max(0, (int)std::floor(xy[2 * p] - 1e-9) - 1 - d.x0);
    const int xb = std::min(d.bw - 1, (int)std::floor(xy[2 * p] + 1e-9) + 2 - d.x0);
    const int ya = std::max(0, (int)std::floor(xy[2 * p + 1] - 1e-9) - 1 - d.y0);
    const int yb = std::min(d.bh - 1, (int)std::floor(xy[2 * p + 1] + 1e-9) + 2 - d.y0);
    for (int ly = ya; ly <= yb; ++ly)
      for (int lx = xa; lx <= xb; ++lx) {
        unsigned char& m = hit[(size_t)ly * d.bw + lx];
        cnt += m == 0;
        m = 1;
      }
  }
  return cnt;
}

// Smallest Cholesky pivot of the perimeter block relative to its largest
// diagonal entry; <= 0 means not positive definite.
double perimeter_conditioning(const std::vector<double>& xy, int n, const ibmlbm_config& c) {
  (void)c;  // the supports of one foil never wrap a periodic axis (checked)
  std::vector<double> M((size_t)n * n);
  // support nodes floor(X) - 1 .. floor(X) + 2 and their kernel weights, per axis
  std::vector<int> f0(2 * n);
  std::vector<double> wt(8 * n);
  for (int p = 0; p < n; ++p)
    for (int d = 0; d < 2; ++d) {
      const double X = xy[2 * p + d];
      f0[2 * p + d] = (int)std::floor(X) - 1;
      for (int k = 0; k < 4; ++k) wt[8 * p + 4 * d + k] = delta_h(f0[2 * p + d] + k - X);
    }
  auto a1 = [&](int p, int q, int d) {
    const int lo = std::max(f0[2 * p + d], f0[2 * q + d]);
    const int hi = std::min(f0[2 * p + d], f0[2 * q + d]) + 3;
    double s = 0.0;
    for (int j = lo; j <= hi; ++j)
      s += wt[8 * p + 4 * d + (j - f0[2 * p + d])] * wt[8 * q + 4 * d + (j - f0[2 * q + d])];
    return s;
  };
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) M[(size_t)p * n + q] = a1(p, q, 0) * a1(p, q, 1);
  double dmax = 0.0;
  for (int p = 0; p < n; ++p) dmax = std::max(dmax, M[(size_t)p * n + p]);
  double pmin = 1e300;
  for (int k = 0; k < n; ++k) {
    double d = M[(size_t)k * n + k];
    for (int j = 0; j < k; ++j) d -= M[(size_t)k * n + j] * M[(size_t)k * n + j];
    if (!(d > 0.0)) return -1.0;
    pmin = std::min(pmin, d);
    const double l = std::sqrt(d);
    M[(size_t)k * n + k] = l;
    for (int i = k + 1; i < n; ++i) {
      double v = M[(size_t)i * n + k];
      for (int j = 0; j < k; ++j) v -= M[(size_t)i * n + j] * M[(size_t)k * n + j];
      M[(size_t)i * n + k] = v / l;
    }
  }
  return pmin / dmax;
}

// Row of the pseudo-inverse of the circulant span factor M_z, with
// M_z[s][s'] = a(s + 1/2, s' + 1/2) on a periodic axis of ns cells.  The
// cosine kernel makes the alternating mode exactly null; eigenvalues below
// 1e-12 of the largest are dropped (minimum-norm solution).
void span_pinv_row(int ns, std::vector<double>& G) {
  // kernel weights of a layer at z = 1/2 on the ns nodes of the periodic
  // axis (support nodes that wrap onto one node add up, as they do for
  // spans shorter than 4); r[j] = a(1/2, j + 1/2) = sum_i I(i) I(i - j)
  std::vector<double> I(ns, 0.0);
  for (int k = 0; k < 4; ++k) {
    const int node = -1 + k;
    I[((node % ns) + ns) % ns] += delta_h(node - 0.5);
  }
  std::vector<double> r(ns, 0.0);
  for (int j = 0; j < ns; ++j)
    for (int i = 0; i < ns; ++i) r[j] += I[i] * I[((i - j) % ns + ns) % ns];
  std::vector<double> lam(ns);
  double lmax = 0.0;
  for (int k = 0; k < ns; ++k) {
    double s = 0.0;
    for (int j = 0; j < ns; ++j) s += r[j] * std::cos(2.0 * M_PI * (double)((long long)j * k % ns) / ns);
    lam[k] = s;
    lmax = std::max(lmax, std::fabs(s));
  }
  G.assign(ns, 0.0);
  for (int j = 0; j < ns; ++j) {
    double s = 0.0;
    for (int k = 0; k < ns; ++k) {
      if (std::fabs(lam[k]) <= 1e-12 * lmax) continue;
      s += std::cos(2.0 * M_PI * (double)((long long)j * k % ns) / ns) / lam[k];
    }
    G[j] = s / ns;
  }
}

int check_wings(const ibmlbm_config& c, int nw, const ibmlbm_wing* w, std::vector<WingGeom>& geo,
                std::string& why) {
  char b[256];
  if (nw < 0 || nw > kMaxWings) { why = "n_wings must be in 0..8"; return IBMLBM_EINVAL; }
  if (nw > 0 && !w) { why = "null wings"; return IBMLBM_EINVAL; }
  geo.assign(nw, WingGeom{});
  if (nw > 0 && c.bc[4] != IBMLBM_BC_PERIODIC) {
    why = "foils are extruded over the span: z must be periodic";
    return IBMLBM_EINVAL;
  }
  if (nw > 0 && marker_span_lds(c.nz) > kMaxLds) {
    int top = c.nz;
    while (top > 1 && marker_span_lds(top) > kMaxLds) --top;
    char b[160];
    snprintf(b, sizeof b, "a span of %d layers does not fit the marker kernels' local memory (at most %d)",
             c.nz, top);
    why = b;
    return IBMLBM_EINVAL;
  }
  for (int k = 0; k < nw; ++k) {
    const ibmlbm_wing& x = w[k];
    if (x.sense != 1.0 && x.sense != -1.0) { why = "sense must be +1 or -1"; return IBMLBM_EINVAL; }
    if (x.alpha_shape < 0 || x.alpha_shape > 2) { why = "unknown alpha shape"; return IBMLBM_EINVAL; }
    if ((x.alpha_shape != IBMLBM_ALPHA_CONST || x.trans_amp != 0.0) && !(x.period_steps > 0.0)) {
      why = "moving foils need period_steps > 0";
      return IBMLBM_EINVAL;
    }
    if (x.pivot_frac < 0.0 || x.pivot_frac > 1.0) { why = "pivot_frac must be in [0, 1]"; return IBMLBM_EINVAL; }
    int rc = wing_geometry(x, geo[k], why);
    if (rc) return rc;
    // every support node floor(X)-1 .. floor(X)+2 stays inside the box in x
    // and y (also on periodic axes: the node boxes of a foil do not wrap)
    const double reach = geo[k].rmax + std::fabs(x.trans_amp);
    // node boxes (support plus one spare cell) stay off Zou-He faces, whose
    // boundary cells are rebuilt after streaming
    const double xlo = c.bc[0] >= IBMLBM_BC_ZH_VELOCITY ? 4.0 : 1.0;
    const double xhi = c.bc[1] >= IBMLBM_BC_ZH_VELOCITY ? 5.0 : 2.0;
    if (x.hinge[0] - reach < xlo || x.hinge[0] + reach >= c.nx - xhi) {
      snprintf(b, sizeof b, "foil %d: marker supports may leave the box along x", k);
      why = b;
      return IBMLBM_EINVAL;
    }
    if (x.hinge[1] - reach < 1.0 || x.hinge[1] + reach >= c.ny - 2.0) {
      snprintf(b, sizeof b, "foil %d: marker supports may leave the box along y", k);
      why = b;
      return IBMLBM_EINVAL;
    }
    geo[k].side = 2 * (int)std::ceil(reach) + 8;
  }
  // sampled over one period of the slowest foil: separation of supports and
  // conditioning of every perimeter block
  double T = 1.0;
  for (int k = 0; k < nw; ++k)
    if (w[k].alpha_shape != IBMLBM_ALPHA_CONST || w[k].trans_amp != 0.0) T = std::max(T, w[k].period_steps);
  const int samples = 97;
  std::vector<std::vector<double>> xy(nw);
  for (int sidx = 0; sidx < samples; ++sidx) {
    const double t = T * sidx / (samples - 1);
    for (int k = 0; k < nw; ++k) {
      perimeter_xy(w[k], geo[k], t, xy[k]);
      if (perimeter_conditioning(xy[k], geo[k].np, c) < 1e-9) {
        snprintf(b, sizeof b, "foil %d: perimeter system (Eq. 18) is singular; raise ds", k);
        why = b;
        return IBMLBM_EINVAL;
      }
    }
    for (int k = 0; k < nw; ++k)
      for (int l = k + 1; l < nw; ++l)
        for (int p = 0; p < geo[k].np; ++p)
          for (int q = 0; q < geo[l].np; ++q) {
            const double dx = std::fabs(xy[k][2 * p] - xy[l][2 * q]);
            const double dy = std::fabs(xy[k][2 * p + 1] - xy[l][2 * q + 1]);
            if (std::max(dx, dy) < 4.5) {
              snprintf(b, sizeof b, "foils %d and %d come within the delta support of each other", k, l);
              why = b;
              return IBMLBM_EINVAL;
            }
          }
    for (int k = 0; k < nw; ++k) {
      // node box at this pose, grown by 3 cells against poses between samples
      WingDev d{};
      node_box(w[k], geo[k], t, c, d);
      const int bw = std::min(d.bw + 3, geo[k].side), bh = std::min(d.bh + 3, geo[k].side);
      geo[k].max_cells = std::max(geo[k].max_cells, bw * bh);
    }
  }
  // local memory of the marker kernels: the perimeter factor block holds the
  // records, the pivot column and row (the matrix itself is in registers)
  // and the support bitmap; the layer block holds the records, the layer's
  // solution, at least one partial spread image of the largest node box and
  // an 8 KB reduction array (markers.hip)
  int maxnp = 0, maxcells = 0;
  for (int k = 0; k < nw; ++k) {
    maxnp = std::max(maxnp, geo[k].np);
    maxcells = std::max(maxcells, geo[k].max_cells);
  }
  int maxside = 0;
  for (int k = 0; k < nw; ++k) maxside = std::max(maxside, geo[k].side);
  const size_t lds_factor = (size_t)(kPwStride + 4) * maxnp * 8 + (size_t)maxside * ((maxside + 31) / 32 + 1) * 4;
  const size_t lds_layer = (size_t)(kPwStride + 6) * maxnp * 8 + 8192 + (size_t)maxcells * 12;
  if (nw > 0 && std::max(lds_factor, lds_layer) > kMaxLds) {
    snprintf(b, sizeof b,
             "%d perimeter markers with a node box of up to %d cells need %zu bytes of the layer kernel's "
             "local memory (limit %zu): reduce the chord or raise ds",
             maxnp, maxcells, std::max(lds_factor, lds_layer), kMaxLds);
    why = b;
    return IBMLBM_EINVAL;
  }
  return IBMLBM_OK;
}

MarkerLayout marker_layout(const ibmlbm_config& c, int nw, const std::vector<WingGeom>& geo,
                           size_t start) {
  MarkerLayout M;
  size_t nref = 0, nG = 0, nMinv = 0;
  for (int k = 0; k < nw; ++k) {
    nref += 2 * geo[k].np;
    nG += c.nz;
    nMinv += (size_t)geo[k].np * geo[k].np;
    M.m_total += geo[k].np * c.nz;
    M.layers += c.nz;
    M.perims += geo[k].np;
  }
  size_t o = align256(start);
  auto take = [&](Region& r, size_t bytes) { r.off = o; r.bytes = bytes; o = align256(o + std::max<size_t>(bytes, 8)); };
  const size_t m = M.m_total;
  take(M.ref, nref * 8);
  take(M.G, nG * 8);
  take(M.Minv, (size_t)kFactorWindow * nMinv * 8);
  take(M.pw, (size_t)kFactorWindow * M.perims * kPwStride * 8);
  for (int k = 0; k < nw; ++k) M.sup_step += 1 + 16 * geo[k].np + geo[k].side * ((geo[k].side + 31) / 32);
  take(M.sup, (size_t)kFactorWindow * M.sup_step * 4);
  M.minv_step = (int)nMinv;
  M.pw_step = M.perims * kPwStride;
  take(M.T, 3 * m * 8);
  take(M.X, 3 * m * 8);
  take(M.U, 3 * m * 8);
  take(M.B, 3 * m * 8);
  take(M.rhoB, m * 8);
  take(M.duB, 3 * m * 8);
  take(M.fpart, 4 * (size_t)M.layers * 8);
  M.band.resize(nw);
  M.corr.resize(nw);
  for (int k = 0; k < nw; ++k) {
    const size_t img = (size_t)geo[k].side * geo[k].side * c.nz * 16;
    take(M.band[k], img);
    take(M.corr[k], img);
  }
  take(M.hist, (size_t)c.history_steps * std::max(nw, 1) * 8 * 8);
  M.end = o;
  return M;
}

void fill_phys(ibmlbm_t h) {
  const ibmlbm_config& c = h->cfg;
  h->phys.omega = (float)(1.0 / c.tau);
  h->phys.guo_k = (float)(1.0 - 0.5 / c.tau);
  for (int d = 0; d < 3; ++d) {
    h->phys.fb[d] = (float)c.body_force[d];
    h->phys.u_in[d] = (float)c.u_in[d];
  }
  h->phys.rho_out = (float)c.rho_out;
}

// Fold the recorded event pairs into the timing sums.
int fold_events(ibmlbm_t h) {
  for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]));
    if (h->ev_kind[k / 2] == 0) {
      h->acc_collide_ms += ms;
      h->acc_collide_n++;
      h->acc_collide_cells += h->ev_cells[k / 2];
    } else {
      h->acc_marker_ms += ms;
    }
  }
  h->ev_used = 0;
  return IBMLBM_OK;
}

// Timing event on stream `st` for the step being enqueued (kind 0: a
// collide launch updating `cells` cells, kind 1: the marker kernels).
int record_event(ibmlbm_t h, hipStream_t st, int kind, bool start, double cells = 0.0) {
  if (!h->timing || h->step % h->timing_every != 0) return IBMLBM_OK;
  if (start) {
    if (h->ev_used + 2 > h->ev.size()) {
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      int rc = fold_events(h);
      if (rc) return rc;
    }
    h->ev_kind[h->ev_used / 2] = kind;
    h->ev_cells[h->ev_used / 2] = cells;
  }
  HIP_TRY(h, hipEventRecord(h->ev[h->ev_used], st));
  h->ev_used++;
  return IBMLBM_OK;
}

// Arguments of step s whose current state is A if cur_A: the parts that
// never change for this handle, then the step's own (state buffers, time,
// window slot, force-history row, node boxes and the grids they imply).
const void* dev_ma(ibmlbm_t h, int slot);

void step_args(ibmlbm_t h, long long s, bool cur_A, CollideArgs& ca, MarkerArgs& ma) {
  const LatticeLayout& L = h->L;
  const ibmlbm_config& c = h->cfg;
  ca = CollideArgs{};
  ma = MarkerArgs{};
  ca.g = h->geo;
  ca.p = h->phys;
  ca.nw = h->nw;
  ca.nxc = L.nxc;
  {
    const float e = (float)delta_h(1.5), d = (float)delta_h(0.5);
    ca.wz[0] = e; ca.wz[1] = d; ca.wz[2] = d; ca.wz[3] = e;
    ma.wz[0] = delta_h(1.5); ma.wz[1] = delta_h(0.5); ma.wz[2] = delta_h(0.5); ma.wz[3] = delta_h(1.5);
  }
  ca.nblocks = L.nblocks;
  ca.nxc_mul = div_mul(L.nxc, (unsigned long long)L.nblocks * kBlockRows);
  ca.ny_mul = div_mul(c.ny, (unsigned long long)c.ny * c.nz);
  ca.mass_part = at<double>(h, L.mass_part);
  ca.flags = reinterpret_cast<int*>(h->sb + L.diag.off + 16);
  void* A = h->ws + L.fA.off;
  void* B = h->ws + L.fB.off;
  ca.src = cur_A ? A : B;
  ca.dst = cur_A ? B : A;
  if (h->nw == 0) return;
  ma.g = h->geo;
  ma.p = h->phys;
  ma.nw = h->nw;
  ma.m_total = h->M.m_total;
  for (int k = 0; k < h->nw; ++k) ma.w[k] = h->wd[k];
  ma.ref = at<double>(h, h->M.ref);
  ma.G = at<double>(h, h->M.G);
  ma.Minv = at<double>(h, h->M.Minv);
  ma.X = at<double>(h, h->M.X);
  ma.U = at<double>(h, h->M.U);
  ma.B = at<double>(h, h->M.B);
  ma.rhoB = at<double>(h, h->M.rhoB);
  ma.duB = at<double>(h, h->M.duB);
  ma.pw = at<double>(h, h->M.pw);
  ma.sup = at<unsigned>(h, h->M.sup);
  ma.sup_step = h->M.sup_step;
  ma.win_args = static_cast<const MarkerArgs*>(dev_ma(h, 0));
  ma.T = at<double>(h, h->M.T);
  ma.fpart = at<double>(h, h->M.fpart);
  ca.fpart = ma.fpart;
  ca.hist = at<double>(h, h->M.hist);
  ca.qS = 0.5 * c.u_ref * c.u_ref * c.area_ref;
  for (int k = 0; k < h->nw; ++k) {
    ca.sense[k] = h->wings[k].sense;
    ca.chord[k] = h->wings[k].chord;
  }
  ma.pw_step = h->M.pw_step;
  ma.minv_step = h->M.minv_step;
  ma.flags = ca.flags;
  ma.win_t0 = h->win_t0;
  ma.slot = (int)(s - h->win_t0);
  ma.t = (double)s;
  for (int k = 0; k < h->nw; ++k) {
    double* q = ma.pose[k];
    wing_pose(ma.w[k], (double)s, q[0], q[1], q[2], q[3], q[4], q[5]);
  }
  ma.src = ca.src;
  ca.hist_row = s % c.history_steps;
  long long band_waves = 0;
  int maxnp = 0, maxcells = 0;
  for (int w = 0; w < h->nw; ++w) {
    node_box(h->wings[w], h->geom[w], (double)s, c, ma.w[w]);
    FoilBox& b = ca.box[w];
    b.x0 = ma.w[w].x0; b.y0 = ma.w[w].y0; b.w = ma.w[w].bw; b.h = ma.w[w].bh;
    b.side = ma.w[w].side;
    b.band = ma.w[w].band;
    b.corr = ma.w[w].corr;
    b.words = ma.w[w].mask_words;
    b.bits = ma.sup + (size_t)ma.slot * ma.sup_step + ma.w[w].sup_off + 1 + 16 * ma.w[w].np;
    ma.w[w].sup_chunks = (support_bound(h->wings[w], h->geom[w], (double)s, ma.w[w]) + 63) / 64;
    band_waves += (long long)ma.w[w].sup_chunks * c.nz;
    maxnp = std::max(maxnp, ma.w[w].np);
    maxcells = std::max(maxcells, ma.w[w].bw * ma.w[w].bh);
  }
  ma.band_blocks = (int)((band_waves + 3) / 4);
  // Layer kernel LDS: the records and the layer's solution, an 8 KiB
  // reduction array, and as many partial spread images (up to 4) as fit in
  // the budget: three blocks per compute unit where one image allows it,
  // else two, else as many as fit.
  const size_t fixed = (size_t)(kPwStride + 6) * maxnp * 8 + 8192;
  const size_t per = (size_t)maxcells * 12;
  const size_t budget = fixed + per <= 53 * 1024 ? 53 * 1024 : (fixed + per <= 80 * 1024 ? 80 * 1024 : 150 * 1024);
  ma.copies = 4;
  while (ma.copies > 1 && fixed + ma.copies * per > budget) --ma.copies;
}

const void* dev_ca(ibmlbm_t h, int slot) {
  return h->sb + h->L.argtab.off + (size_t)slot * sizeof(CollideArgs);
}
const void* dev_ma(ibmlbm_t h, int slot) {
  return h->sb + h->L.argtab.off + (size_t)kFactorWindow * sizeof(CollideArgs) +
         (size_t)slot * sizeof(MarkerArgs);
}

// Start a window at step s0: the arguments of its kFactorWindow steps are
// made on the host and uploaded in one copy, enqueued on the handle's
// stream ahead of the window's launches.
int fill_window(ibmlbm_t h, long long s0) {
  h->win_t0 = s0;
  h->wca.resize(kFactorWindow);
  h->wma.resize(kFactorWindow);
  for (int k = 0; k < kFactorWindow; ++k)
    step_args(h, s0 + k, h->cur_is_A == ((k & 1) == 0), h->wca[k], h->wma[k]);
  if (h->pin_pending) HIP_TRY(h, hipEventSynchronize(h->pin_ev));
  char* dev = h->sb + h->L.argtab.off;
  const size_t cb = (size_t)kFactorWindow * sizeof(CollideArgs), mb = (size_t)kFactorWindow * sizeof(MarkerArgs);
  if (h->pin) {
    char* pin = static_cast<char*>(h->pin);
    std::memcpy(pin, h->wca.data(), cb);
    std::memcpy(pin + cb, h->wma.data(), mb);
    HIP_TRY(h, hipMemcpyAsync(dev, pin, cb + mb, hipMemcpyHostToDevice, h->stream));
  } else {
    // no pinned staging (ibmlbm_create_noalloc): straight from the host
    // copies, which are not touched again before the event below completes
    HIP_TRY(h, hipMemcpyAsync(dev, h->wca.data(), cb, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(dev + cb, h->wma.data(), mb, hipMemcpyHostToDevice, h->stream));
  }
  HIP_TRY(h, hipEventRecord(h->pin_ev, h->stream));
  h->pin_pending = true;
  return IBMLBM_OK;
}

bool has_force(const ibmlbm_config& c) {
  return c.body_force[0] != 0.0 || c.body_force[1] != 0.0 || c.body_force[2] != 0.0;
}

// Zou-He x faces: their cells are rebuilt inside the collide kernel, by its
// instantiation for such solves.
bool has_zou_he(const ibmlbm_config& c) {
  return c.bc[0] >= IBMLBM_BC_ZH_VELOCITY || c.bc[1] >= IBMLBM_BC_ZH_VELOCITY;
}

// `steps` time steps of every handle in hs (one stream).  Each stage of a
// step is one grouped launch over the handles that share its kernel
// instantiation, so small solves fill the device together and each solve
// runs the same code as alone.
int run_steps(ibmlbm_t* hs, int n, int steps) {
  hipStream_t st = hs[0]->stream;
  const bool timed = n == 1;
  std::vector<const MarkerArgs*> mh;
  std::vector<const CollideArgs*> chh;
  std::vector<const void*> dv;
  for (int k = 0; k < steps; ++k) {
    // windows that start at this step; their factor launch
    mh.clear();
    dv.clear();
    for (int j = 0; j < n; ++j) {
      ibmlbm_t h = hs[j];
      const long long s = h->step;
      if (h->win_t0 < 0 || s < h->win_t0 || s >= h->win_t0 + kFactorWindow) {
        int rc = fill_window(h, s);
        if (rc) return rc;
        if (h->nw > 0) {
          mh.push_back(&h->wma[0]);
          dv.push_back(dev_ma(h, 0));
        }
      }
    }
    bool any_ibm = false;
    for (int j = 0; j < n; ++j) any_ibm = any_ibm || hs[j]->nw > 0;
    if (timed && any_ibm) {
      int rc = record_event(hs[0], st, 1, true);
      if (rc) return rc;
    }
    if (!mh.empty()) {
      hipError_t e = launch_factor(mh.data(), dv.data(), (int)mh.size(), kFactorWindow, st);
      if (e != hipSuccess) return fail(hs[0], IBMLBM_EDEVICE, "factor launch: %s", hipGetErrorString(e));
    }
    // marker kernels, grouped by storage
    for (int sto = 0; sto < 3; ++sto) {
      mh.clear();
      dv.clear();
      for (int j = 0; j < n; ++j) {
        ibmlbm_t h = hs[j];
        if (h->nw == 0 || h->cfg.storage != sto) continue;
        const int slot = (int)(h->step - h->win_t0);
        mh.push_back(&h->wma[slot]);
        dv.push_back(dev_ma(h, slot));
      }
      if (mh.empty()) continue;
      hipError_t e = launch_markers(sto, mh.data(), dv.data(), (int)mh.size(), st);
      if (e != hipSuccess) return fail(hs[0], IBMLBM_EDEVICE, "marker launch: %s", hipGetErrorString(e));
    }
    if (timed && any_ibm) {
      int rc = record_event(hs[0], st, 1, false);
      if (rc) return rc;
    }
    // collide, grouped by (storage, foils, body force, check step)
    if (timed) {
      int rc = record_event(hs[0], st, 0, true, (double)hs[0]->L.N);
      if (rc) return rc;
    }
    for (int key = 0; key < 48; ++key) {
      const int sto = key >> 4;
      const bool zh = key & 8, ibm = key & 4, force = key & 2, check = key & 1;
      chh.clear();
      dv.clear();
      for (int j = 0; j < n; ++j) {
        ibmlbm_t h = hs[j];
        const ibmlbm_config& c = h->cfg;
        const bool ck = c.check_interval > 0 && ((h->step + 1) % c.check_interval == 0);
        if (c.storage != sto || (h->nw > 0) != ibm || has_force(c) != force || ck != check ||
            has_zou_he(c) != zh)
          continue;
        const int slot = (int)(h->step - h->win_t0);
        chh.push_back(&h->wca[slot]);
        dv.push_back(dev_ca(h, slot));
      }
      if (chh.empty()) continue;
      hipError_t e = launch_collide(sto, ibm, force, check, zh, chh.data(), dv.data(), (int)chh.size(), st);
      if (e != hipSuccess) return fail(hs[0], IBMLBM_EDEVICE, "collide launch: %s", hipGetErrorString(e));
    }
    if (timed) {
      int rc = record_event(hs[0], st, 0, false);
      if (rc) return rc;
    }
    for (int j = 0; j < n; ++j) {
      ibmlbm_t h = hs[j];
      const ibmlbm_config& c = h->cfg;
      const long long s = h->step;
      if (c.check_interval > 0 && ((s + 1) % c.check_interval == 0))
        HIP_TRY(h, launch_mass_reduce(at<double>(h, h->L.mass_part), h->L.nblocks,
                                      (double)h->L.N,
                                      reinterpret_cast<double*>(h->sb + h->L.diag.off), s + 1, st));
      h->cur_is_A = !h->cur_is_A;
      h->step = s + 1;
      if (h->nw > 0) h->markers_valid = true;
    }
  }
  return IBMLBM_OK;
}

// Handle of a solve.  noalloc: the caller's buffer holds the two lattice
// states only; every other region comes from this device's static scratch
// (scratch.hip), and no pinned staging buffer is made.
int create_handle(const ibmlbm_config* cfg, void* dev_buf, size_t bytes, void* hip_stream, ibmlbm_t* out,
                  bool noalloc) {
  if (!out) return fail(nullptr, IBMLBM_EINVAL, "null output handle");
  *out = nullptr;
  std::string why;
  int rc = validate_config(cfg, why);
  if (rc) return fail(nullptr, rc, "%s", why.c_str());
  if (!dev_buf) return fail(nullptr, IBMLBM_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(nullptr, IBMLBM_EINVAL, "workspace must be 256-byte aligned");
  LatticeLayout L = lattice_layout(cfg, noalloc);
  const size_t need = noalloc ? L.state_end : L.end;
  if (bytes < need) return fail(nullptr, IBMLBM_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, need);
  char* sb = static_cast<char*>(dev_buf);
  size_t sb_bytes = bytes;
  if (noalloc) {
    int dev = 0;
    void* p = nullptr;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = scratch_address(dev, &p);
    if (e != hipSuccess) return fail(nullptr, IBMLBM_EDEVICE, "static scratch: %s", hipGetErrorString(e));
    if (L.end > kScratchBytes)
      return fail(nullptr, IBMLBM_ENOMEM, "the lattice needs %zu bytes of scratch, beyond the static scratch of %zu bytes",
                  L.end, kScratchBytes);
    sb = static_cast<char*>(p);
    sb_bytes = kScratchBytes;
  }
  ibmlbm_t h = new ibmlbm_s();
  h->cfg = *cfg;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(dev_buf);
  h->ws_bytes = bytes;
  h->sb = sb;
  h->sb_bytes = sb_bytes;
  h->noalloc = noalloc;
  h->L = L;
  h->geo.nx = cfg->nx;
  h->geo.ny = cfg->ny;
  h->geo.nz = cfg->nz;
  h->geo.px = L.px;
  h->geo.ps = L.ps;
  h->geo.goff = (long long)L.goff;
  h->geo.yper = cfg->bc[2] == IBMLBM_BC_PERIODIC;
  h->geo.zper = cfg->bc[4] == IBMLBM_BC_PERIODIC;
  h->geo.bclo = cfg->bc[0];
  h->geo.bchi = cfg->bc[1];
  fill_phys(h);
  // mass, step and flags start at zero (the static scratch keeps the last
  // solve's contents)
  hipError_t e = hipMemsetAsync(h->sb + L.diag.off, 0, L.diag.bytes, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && !noalloc) e = hipHostMalloc(&h->pin, L.argtab.bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->pin_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    int r = fail(nullptr, IBMLBM_EDEVICE, "create failed: %s", hipGetErrorString(e));
    ibmlbm_destroy(h);
    return r;
  }
  *out = h;
  return IBMLBM_OK;
}

}  // namespace

// ================================================================== C ABI ==
extern "C" {

size_t ibmlbm_workspace_bytes(const ibmlbm_config* cfg, int32_t n_wings, const ibmlbm_wing* wings) {
  std::string why;
  if (validate_config(cfg, why)) { g_err = why; return 0; }
  LatticeLayout L = lattice_layout(cfg);
  if (n_wings == 0) return L.end;
  std::vector<WingGeom> geo;
  if (check_wings(*cfg, n_wings, wings, geo, why)) { g_err = why; return 0; }
  return marker_layout(*cfg, n_wings, geo, L.end).end;
}

int ibmlbm_create(const ibmlbm_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                  ibmlbm_t* out) {
  return create_handle(cfg, dev_workspace, bytes, hip_stream, out, false);
}

int ibmlbm_create_noalloc(const ibmlbm_config* cfg, void* dev_state, size_t bytes, void* hip_stream,
                          ibmlbm_t* out) {
  return create_handle(cfg, dev_state, bytes, hip_stream, out, true);
}

int ibmlbm_init_fields(ibmlbm_t h, const double* rho, const double* u, const double* fdist, int64_t step0) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (step0 < 0) return fail(h, IBMLBM_EINVAL, "step0 must be >= 0");
  const LatticeLayout& L = h->L;
  const size_t N = L.N;
  h->cur_is_A = true;
  void* dst = h->ws + L.fA.off;
  if (fdist) {
    // pack f_i - w_i into the padded layout on the host
    const double w[kQ] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    std::vector<unsigned char> host(L.total * L.es, 0);
    const int nx = h->cfg.nx, ny = h->cfg.ny, nz = h->cfg.nz;
    for (int q = 0; q < kQ; ++q)
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x) {
            const size_t cell = ((size_t)z * ny + y) * nx + x;
            const float v = (float)(fdist[(size_t)q * N + cell] - w[q]);
            const size_t idx = (((size_t)(z * ny + y) + 1) * kQ + q) * L.px + x;
            if (L.es == 4) {
              std::memcpy(&host[idx * 4], &v, 4);
            } else if (h->cfg.storage == IBMLBM_FP16_DEV) {
              _Float16 hv = (_Float16)(v * kF16Scale);
              std::memcpy(&host[idx * 2], &hv, 2);
            } else {
              uint32_t u32;
              std::memcpy(&u32, &v, 4);
              u32 += 0x7fffu + ((u32 >> 16) & 1u);
              const uint16_t b16 = (uint16_t)(u32 >> 16);
              std::memcpy(&host[idx * 2], &b16, 2);
            }
          }
    HIP_TRY(h, hipMemcpyAsync(dst, host.data(), host.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  } else {
    // stage FP64 rho and u in the other state buffer (free between steps)
    double* stage = reinterpret_cast<double*>(h->ws + L.fB.off);
    if ((rho ? N : 0) * 8 + (u ? 3 * N : 0) * 8 > L.fB.bytes)
      return fail(h, IBMLBM_ENOMEM, "staging area too small");
    double* drho = rho ? stage : nullptr;
    double* du = u ? stage + (rho ? N : 0) : nullptr;
    if (rho) HIP_TRY(h, hipMemcpyAsync(drho, rho, N * 8, hipMemcpyHostToDevice, h->stream));
    if (u) HIP_TRY(h, hipMemcpyAsync(du, u, 3 * N * 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, launch_init_eq(h->cfg.storage, h->geo, drho, du, dst, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  HIP_TRY(h, launch_ghost(h->cfg.storage, h->geo, h->phys, dst, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->step = step0;
  h->initialized = true;
  h->markers_valid = false;
  h->win_t0 = -1;
  return IBMLBM_OK;
}

int ibmlbm_set_kinematics(ibmlbm_t h, int32_t n_wings, const ibmlbm_wing* wings) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  std::string why;
  std::vector<WingGeom> geo;
  int rc = check_wings(h->cfg, n_wings, wings, geo, why);
  if (rc) return fail(h, rc, "%s", why.c_str());
  MarkerLayout M = marker_layout(h->cfg, n_wings, geo, h->L.end);
  if (n_wings > 0 && M.end > h->sb_bytes) {
    if (h->noalloc)
      return fail(h, IBMLBM_ENOMEM, "the markers need %zu bytes of scratch, beyond the static scratch of %zu bytes",
                  M.end, h->sb_bytes);
    return fail(h, IBMLBM_ENOMEM, "workspace of %zu bytes < %zu needed for the markers", h->ws_bytes, M.end);
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->nw = n_wings;
  h->geom = geo;
  h->M = M;
  h->markers_valid = false;
  h->win_t0 = -1;
  if (n_wings == 0) return IBMLBM_OK;
  std::vector<double> ref, G;
  int moff = 0, roff = 0, goff = 0, moff2 = 0, pwoff = 0, loff = 0, supoff = 0;
  for (int k = 0; k < n_wings; ++k) {
    const ibmlbm_wing& w = wings[k];
    h->wings[k] = w;
    WingDev& d = h->wd[k];
    d.np = geo[k].np;
    d.ns = h->cfg.nz;
    d.moff = moff;
    d.ref_off = roff;
    d.g_off = goff;
    d.minv_off = moff2;
    d.pw_off = pwoff;
    d.sup_off = supoff;
    d.mask_words = (geo[k].side + 31) / 32;
    d.c_off = 3 * moff;
    d.layer_off = loff;
    d.side = geo[k].side;
    d.band = at<float4>(h, M.band[k]);
    d.corr = at<float4>(h, M.corr[k]);
    d.shape = w.alpha_shape;
    d.hinge0[0] = w.hinge[0];
    d.hinge0[1] = w.hinge[1];
    d.theta0 = w.theta0;
    d.sense = w.sense;
    d.mean = w.alpha_mean;
    d.amp = w.alpha_amp;
    d.period = w.period_steps > 0.0 ? w.period_steps : 1.0;
    d.phase = w.phase;
    d.tamp = w.trans_amp;
    d.tang = w.trans_angle;
    d.dA = geo[k].ds * 1.0;
    d.chord = w.chord;
    ref.insert(ref.end(), geo[k].ref.begin(), geo[k].ref.end());
    std::vector<double> g;
    span_pinv_row(h->cfg.nz, g);
    G.insert(G.end(), g.begin(), g.end());
    moff += d.np * d.ns;
    roff += 2 * d.np;
    goff += d.ns;
    moff2 += d.np * d.np;
    pwoff += kPwStride * d.np;
    supoff += 1 + 16 * d.np + d.side * d.mask_words;
    loff += d.ns;
  }
  HIP_TRY(h, hipMemcpyAsync(h->sb + M.ref.off, ref.data(), ref.size() * 8, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->sb + M.G.off, G.data(), G.size() * 8, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemsetAsync(h->sb + M.hist.off, 0, M.hist.bytes, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return IBMLBM_OK;
}

int ibmlbm_step(ibmlbm_t h, int32_t n) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (!h->initialized) return fail(h, IBMLBM_ESTATE, "init_fields must be called before step");
  if (n < 0) return fail(h, IBMLBM_EINVAL, "negative step count");
  return run_steps(&h, 1, n);
}

int ibmlbm_step_batch(ibmlbm_t* hs, int32_t n_handles, int32_t n) {
  if (!hs || n_handles < 1 || n_handles > kMaxGroup)
    return fail(nullptr, IBMLBM_EINVAL, "step_batch takes 1..%d handles", kMaxGroup);
  if (n < 0) return fail(nullptr, IBMLBM_EINVAL, "negative step count");
  for (int j = 0; j < n_handles; ++j) {
    if (!hs[j]) return fail(nullptr, IBMLBM_EINVAL, "null handle %d", j);
    if (!hs[j]->initialized) return fail(hs[j], IBMLBM_ESTATE, "handle %d: init_fields must be called before step", j);
    if (hs[j]->stream != hs[0]->stream)
      return fail(nullptr, IBMLBM_EINVAL, "handles of one batch must share one stream");
    for (int k = 0; k < j; ++k)
      if (hs[k] == hs[j]) return fail(nullptr, IBMLBM_EINVAL, "handle %d appears twice", j);
  }
  return run_steps(hs, n_handles, n);
}

int64_t ibmlbm_step_count(ibmlbm_t h) { return h ? h->step : -1; }

int ibmlbm_forces(ibmlbm_t h, int64_t first, int64_t count, double* out) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (count < 0 || first < 0 || (count > 0 && !out)) return fail(h, IBMLBM_EINVAL, "bad range or null output");
  if (h->nw == 0) return count == 0 ? IBMLBM_OK : fail(h, IBMLBM_ESTATE, "no foils");
  const long long H = h->cfg.history_steps;
  if (first + count > h->step || first < h->step - H)
    return fail(h, IBMLBM_ERANGE, "history rows [%lld, %lld) not held (have [%lld, %lld))",
                (long long)first, (long long)(first + count), (long long)std::max(0LL, h->step - H),
                (long long)h->step);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  int flags = 0;
  HIP_TRY(h, hipMemcpy(&flags, h->sb + h->L.diag.off + 16, 4, hipMemcpyDeviceToHost));
  const size_t row = (size_t)h->nw * 8;
  const double* hist = at<double>(h, h->M.hist);
  // the rows form at most two contiguous runs of the ring
  for (long long k = 0; k < count;) {
    const long long r = (first + k) % H;
    const long long run = std::min<long long>(count - k, H - r);
    HIP_TRY(h, hipMemcpy(out + k * row, hist + r * row, (size_t)run * row * 8, hipMemcpyDeviceToHost));
    k += run;
  }
  if (flags & 4) return fail(h, IBMLBM_EDEVICE, "a foil's support nodes outnumbered the band grid sized for them");
  if (flags & 2) return fail(h, IBMLBM_EDIVERGED, "a perimeter system became singular");
  if (flags & 1) return fail(h, IBMLBM_EDIVERGED, "non-finite density seen on a check step");
  return IBMLBM_OK;
}

int ibmlbm_fields(ibmlbm_t h, int32_t which, double* out) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (!out) return fail(h, IBMLBM_EINVAL, "null output");
  if (!h->initialized) return fail(h, IBMLBM_ESTATE, "fields before init_fields");
  const LatticeLayout& L = h->L;
  const size_t N = L.N;
  const int nx = h->cfg.nx, ny = h->cfg.ny, nz = h->cfg.nz;
  if (which == IBMLBM_FIELD_RHO || which == IBMLBM_FIELD_U) {
    float* scratch = static_cast<float*>(next_state(h));
    HIP_TRY(h, launch_moments(h->cfg.storage, h->geo, h->phys, cur_state(h), scratch, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::vector<float> host(4 * N);
    HIP_TRY(h, hipMemcpy(host.data(), scratch, 4 * N * sizeof(float), hipMemcpyDeviceToHost));
    if (which == IBMLBM_FIELD_RHO)
      for (size_t i = 0; i < N; ++i) out[i] = host[i];
    else
      for (size_t i = 0; i < 3 * N; ++i) out[i] = host[N + i];
    return IBMLBM_OK;
  }
  if (which != IBMLBM_FIELD_FDIST) return fail(h, IBMLBM_EINVAL, "unknown field %d", which);
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  std::vector<unsigned char> host(L.total * L.es);
  HIP_TRY(h, hipMemcpy(host.data(), cur_state(h), host.size(), hipMemcpyDeviceToHost));
  const double w[kQ] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (int q = 0; q < kQ; ++q)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const size_t cell = ((size_t)z * ny + y) * nx + x;
          const size_t idx = (((size_t)(z * ny + y) + 1) * kQ + q) * L.px + x;
          float v;
          if (L.es == 4) {
            std::memcpy(&v, &host[idx * 4], 4);
          } else if (h->cfg.storage == IBMLBM_FP16_DEV) {
            _Float16 hv;
            std::memcpy(&hv, &host[idx * 2], 2);
            v = (float)hv * kF16Unscale;
          } else {
            uint16_t b16;
            std::memcpy(&b16, &host[idx * 2], 2);
            const uint32_t u32 = (uint32_t)b16 << 16;
            std::memcpy(&v, &u32, 4);
          }
          out[(size_t)q * N + cell] = w[q] + (double)v;
        }
  return IBMLBM_OK;
}

int32_t ibmlbm_marker_count(ibmlbm_t h) { return h ? h->M.m_total * (h->nw > 0) : 0; }

int ibmlbm_markers(ibmlbm_t h, int32_t which, double* out) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (!out) return fail(h, IBMLBM_EINVAL, "null output");
  if (h->nw == 0) return fail(h, IBMLBM_ESTATE, "no foils");
  const size_t m = h->M.m_total;
  if (which == IBMLBM_MARKER_DA) {
    for (int k = 0; k < h->nw; ++k)
      for (int i = 0; i < h->wd[k].np * h->wd[k].ns; ++i) out[h->wd[k].moff + i] = h->wd[k].dA;
    return IBMLBM_OK;
  }
  if (!h->markers_valid) return fail(h, IBMLBM_ESTATE, "no completed step with markers yet");
  const Region* r = nullptr;
  size_t count = 3 * m;
  switch (which) {
    case IBMLBM_MARKER_X: r = &h->M.X; break;
    case IBMLBM_MARKER_U: r = &h->M.U; break;
    case IBMLBM_MARKER_RHS: r = &h->M.B; break;
    case IBMLBM_MARKER_DU: r = &h->M.duB; break;
    case IBMLBM_MARKER_RHO: r = &h->M.rhoB; count = m; break;
    default: return fail(h, IBMLBM_EINVAL, "unknown marker field %d", which);
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemcpy(out, h->sb + r->off, count * 8, hipMemcpyDeviceToHost));
  return IBMLBM_OK;
}

int ibmlbm_mass(ibmlbm_t h, int64_t* step, double* mass) {
  if (!h || !step || !mass) return fail(h, IBMLBM_EINVAL, "null argument");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  double d[2];
  int flags = 0;
  HIP_TRY(h, hipMemcpy(d, h->sb + h->L.diag.off, 16, hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(&flags, h->sb + h->L.diag.off + 16, 4, hipMemcpyDeviceToHost));
  *mass = d[0];
  *step = d[1] > 0.0 ? (int64_t)d[1] : -1;
  if (flags & 1) return fail(h, IBMLBM_EDIVERGED, "non-finite density seen on a check step");
  return IBMLBM_OK;
}

int ibmlbm_set_stream(ibmlbm_t h, void* hip_stream) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->pin_pending = false;   // the last upload was read before the synchronisation
  return IBMLBM_OK;
}

int ibmlbm_timing(ibmlbm_t h, int32_t enable) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  if (enable > 0 && h->ev.empty()) {
    const int pairs = 4096;
    h->ev.resize(2 * pairs);
    h->ev_kind.assign(pairs, 0);
    h->ev_cells.assign(pairs, 0.0);
    // no system-scope fence: the events only time kernels on this device
    for (auto& e : h->ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  h->timing = enable > 0;
  h->timing_every = enable > 0 ? enable : 1;
  return IBMLBM_OK;
}

int ibmlbm_read_timing(ibmlbm_t h, double* collide_ms, int64_t* collide_launches,
                       double* collide_cells, double* marker_ms) {
  if (!h) return fail(nullptr, IBMLBM_EINVAL, "null handle");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  int rc = fold_events(h);
  if (rc) return rc;
  if (collide_ms) *collide_ms = h->acc_collide_ms;
  if (collide_launches) *collide_launches = h->acc_collide_n;
  if (collide_cells) *collide_cells = h->acc_collide_cells;
  if (marker_ms) *marker_ms = h->acc_marker_ms;
  h->acc_collide_ms = h->acc_marker_ms = h->acc_collide_cells = 0.0;
  h->acc_collide_n = 0;
  return IBMLBM_OK;
}

int32_t ibmlbm_bytes_per_cell(ibmlbm_t h) { return h ? 2 * kQ * h->L.es : 0; }

int ibmlbm_destroy(ibmlbm_t h) {
  if (!h) return IBMLBM_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  for (auto& ev : h->ev) (void)hipEventDestroy(ev);
  if (h->pin_ev) (void)hipEventDestroy(h->pin_ev);
  if (h->pin) (void)hipHostFree(h->pin);
  delete h;
  if (e != hipSuccess) return fail(nullptr, IBMLBM_EDEVICE, "stream error at destroy: %s", hipGetErrorString(e));
  return IBMLBM_OK;
}

const char* ibmlbm_last_error(ibmlbm_t h) { return h ? h->err.c_str() : g_err.c_str(); }

int ibmlbm_lattice_params(double Re, double J, double f, double chord, double kappa, double* tau,
                          double* u_inf, double* u_tip, double* period_steps) {
  if (!(Re > 0.0) || !(f > 0.0) || !(chord > 0.0) || !(kappa > 0.0) || J < 0.0)
    return fail(nullptr, IBMLBM_EINVAL, "Re, f, chord, kappa must be > 0 and J >= 0");
  const double Phi = 2.0 * M_PI / 3.0;
  const double ut = kappa * f;
  const double nu = ut * chord / Re;
  if (tau) *tau = 3.0 * nu + 0.5;
  if (u_inf) *u_inf = J * ut;
  if (u_tip) *u_tip = ut;
  if (period_steps) *period_steps = 2.0 * Phi * chord / ut;
  return IBMLBM_OK;
}

int ibmlbm_plate_params(double Re, double u_inf, double chord, double* tau) {
  if (!(Re > 0.0) || !(u_inf > 0.0) || !(chord > 0.0))
    return fail(nullptr, IBMLBM_EINVAL, "Re, u_inf and chord must be > 0");
  const double nu = u_inf * chord / Re;
  if (tau) *tau = 3.0 * nu + 0.5;
  return IBMLBM_OK;
}

int ibmlbm_figure_eight_params(double Re, double u_tip, double chord, double a0, double* tau,
                               double* period_steps) {
  if (!(Re > 0.0) || !(u_tip > 0.0) || !(chord > 0.0) || !(a0 > 0.0))
    return fail(nullptr, IBMLBM_EINVAL, "Re, u_tip, chord and A0 must be > 0");
  const double nu = u_tip * chord / Re;
  if (tau) *tau = 3.0 * nu + 0.5;
  if (period_steps) *period_steps = M_PI * a0 / u_tip;
  return IBMLBM_OK;
}

}  // extern "C"
