// orc.cpp -- FP64 CPU reference for the Yee FDTD hot path (test infrastructure).
//
// Plain triple loops, one per field component, written from the equations of
// Section 2.1 of the paper (eqs. 2-5), the CPML and thin wire of Sections
// 2.2-2.3, the Debye media of Section 2.4, the oblique thin wire the paper
// names in Section 2.3, and the readings stated below.  No tiling, no fusion,
// no reordering beyond "all H, then the oblique-wire currents, then all E,
// then the sources and oblique-wire injection, then the Debye currents, then
// the probes" within a step.  OpenMP
// splits the outer k loop of each component update; every update reads only
// values that the same loop does not write, so the result is independent of
// the thread count.
//
// Parity unpinned (no closed form or published value to check against): the
// exact thin-wire factor of the cited wire papers and their adaptation to
// Debye media; the wires are pinned only at the method's accuracy against
// transmission-line closed forms (in vacuum and in Debye soil).  The
// interface averaging of eps, sigma, mu and pole increments is pinned by
// mirror, rotation, resistor- and capacitor-network and layered-cavity
// tests.  The oblique wire's equivalent radius (the same r0 as the axis
// wires), its vacuum L' and C' and its junctions are a reading (the paper
// names the model, not its equations); its transfer weights, telegraph step,
// charge bookkeeping and junction update are pinned, and so is the line it
// forms (speed c0; impedance within the accuracy stated at its test).
#include "orc.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include <omp.h>

namespace {

const double kPi = 3.14159265358979323846;
const double kMu0 = 4.0e-7 * kPi;                 // H/m
const double kC0 = 299792458.0;                   // m/s
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);    // F/m
const double kEta0 = std::sqrt(kMu0 / kEps0);     // ohm

// A 3D array of doubles with its own extent (x fastest).
struct A3 {
  int n0 = 0, n1 = 0, n2 = 0;
  std::vector<double> v;
  void init(int a, int b, int c, double x = 0.0) {
    n0 = a; n1 = b; n2 = c;
    v.assign((size_t)a * b * c, x);
  }
  double& operator()(int i, int j, int k) { return v[((size_t)k * n1 + j) * n0 + i]; }
  bool in(int i, int j, int k) const {
    return i >= 0 && j >= 0 && k >= 0 && i < n0 && j < n1 && k < n2;
  }
};

struct Wire { int axis, p[3], n; double radius; };
struct Source { int axis, p[3]; std::vector<double> amps; };
struct Lumped { int kind, axis, p[3]; double value; };
struct Probe { int kind, axis, p[3], n; std::vector<double> rec; };
// Oblique thin wire: end points A, B in cells, unit direction t, segment
// length dl (cells), n segments; per-unit-length inductance and capacitance;
// segment currents I (n), end-point charges per unit length q (n + 1), an
// optional hard-driven segment and an optional recorded segment.
struct OWire {
  double A[3], t[3], dl, Lp, Cp;
  int n, src, rec;
  int junc[2] = {-1, -1};  // junction of the start (0) and end (1) node, -1: open end
  std::vector<double> amps, I, q, rec_v;
};
// Junction: end nodes of several oblique wires that meet at one point.
struct OJunction { std::vector<int> wire, end; };

}  // namespace

struct orc_sim {
  orc_params P{};
  double dx = 0, dt = 0;
  int N[3] = {0, 0, 0};
  bool finalized = false;
  long step = 0;
  std::string err;

  // per-cell materials (x fastest)
  std::vector<double> c_eps, c_sig, c_mu;
  std::vector<uint8_t> c_mat;       // material ids of the last set_materials
  int n_mat = 0;
  std::vector<Wire> wires;
  std::vector<Source> srcs;
  std::vector<Lumped> lumped;
  std::vector<Probe> probes;
  std::vector<OWire> owires;
  std::vector<OJunction> ojunc;

  // fields at their natural Yee extents
  A3 E[3], H[3];
  // per-edge / per-face material and coefficients
  A3 eps[3], sig[3], mu[3], Ca[3], Cb[3], Db[3];
  std::vector<char> pec[3];         // wire axial edges (perfect conductor)
  std::vector<char> emod[3], hmod[3];  // already modified by an earlier wire
  // CPML: psi[c][u] for component c (0..2 E, 3..5 H) and derivative axis u
  A3 psi[6][3];
  // Debye media (ADE): pole time constants, eps0 * delta-eps per cell and
  // pole (set-up), per E edge (built, then freed), and per E edge the
  // polarisation current J, its update factor beta, the factor gam of J in
  // the E update, and E before the step (for the J update)
  int npole = 0;
  double tau[4] = {0, 0, 0, 0}, kp[4] = {0, 0, 0, 0};
  std::vector<double> c_deps;       // [cell * npole + p]
  A3 deps[3][4], J[3][4], Jbeta[3][4], Jgam[3][4], Eprev[3];
  std::vector<double> be[3], ce[3], ike[3], bh[3], ch[3], ikh[3];
};

namespace {

int fail(orc_sim* s, int code, const std::string& msg) {
  s->err = msg;
  return code;
}

// Natural extents: E_a has N_a entries along a and N_b + 1 along the others;
// H_a has N_a + 1 along a and N_b along the others.
void e_extent(const orc_sim* s, int a, int ext[3]) {
  for (int b = 0; b < 3; ++b) ext[b] = (b == a) ? s->N[b] : s->N[b] + 1;
}
void h_extent(const orc_sim* s, int a, int ext[3]) {
  for (int b = 0; b < 3; ++b) ext[b] = (b == a) ? s->N[b] + 1 : s->N[b];
}

size_t cell_index(const orc_sim* s, int i, int j, int k) {
  return ((size_t)k * s->N[1] + j) * s->N[0] + i;
}

bool cell_in(const orc_sim* s, const int c[3]) {
  for (int b = 0; b < 3; ++b)
    if (c[b] < 0 || c[b] >= s->N[b]) return false;
  return true;
}

// Is the E_a edge at node p one that the update touches?  Tangential E on the
// six outer faces is held at zero (perfect conductor walls).
bool e_interior(const orc_sim* s, int a, const int p[3]) {
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      if (p[b] < 0 || p[b] >= s->N[b]) return false;
    } else {
      if (p[b] < 1 || p[b] > s->N[b] - 1) return false;
    }
  }
  return true;
}

// Interface rules (the paper is silent): eps and sigma of an edge are the
// arithmetic mean over the in-domain cells that share the edge (tangential E
// is continuous across interfaces, so the cells act in parallel); mu of a
// face is the harmonic mean of the cells on either side (normal B is
// continuous, so they act in series).
void build_materials(orc_sim* s) {
  for (int a = 0; a < 3; ++a) {
    int ext[3];
    e_extent(s, a, ext);
    s->eps[a].init(ext[0], ext[1], ext[2], kEps0);
    s->sig[a].init(ext[0], ext[1], ext[2], 0.0);
    for (int d = 0; d < s->npole; ++d) s->deps[a][d].init(ext[0], ext[1], ext[2], 0.0);
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          const int p[3] = {i, j, k};
          double se = 0, ss = 0, sd[4] = {0, 0, 0, 0};
          int cnt = 0;
          for (int db = -1; db <= 0; ++db)
            for (int dc = -1; dc <= 0; ++dc) {
              int q[3] = {p[0], p[1], p[2]};
              q[b] += db;
              q[c] += dc;
              if (!cell_in(s, q)) continue;
              const size_t ci = cell_index(s, q[0], q[1], q[2]);
              se += s->c_eps[ci];
              ss += s->c_sig[ci];
              for (int d = 0; d < s->npole; ++d) sd[d] += s->c_deps[ci * s->npole + d];
              ++cnt;
            }
          if (cnt) {
            s->eps[a](i, j, k) = se / cnt;
            s->sig[a](i, j, k) = ss / cnt;
            for (int d = 0; d < s->npole; ++d) s->deps[a][d](i, j, k) = sd[d] / cnt;
          }
        }
    h_extent(s, a, ext);
    s->mu[a].init(ext[0], ext[1], ext[2], kMu0);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          double inv = 0;
          int cnt = 0;
          for (int da = -1; da <= 0; ++da) {
            int q[3] = {i, j, k};
            q[a] += da;
            if (!cell_in(s, q)) continue;
            inv += 1.0 / s->c_mu[cell_index(s, q[0], q[1], q[2])];
            ++cnt;
          }
          if (cnt) s->mu[a](i, j, k) = cnt / inv;
        }
    s->pec[a].assign(s->E[a].v.size(), 0);
    s->emod[a].assign(s->E[a].v.size(), 0);
    s->hmod[a].assign(s->H[a].v.size(), 0);
  }
}

// Thin wire (Section 2.3, the assigned-parameter modification model).  The
// paper cites the model without formulas; the reading used here:
//  * the wire's own (axial) edges are perfect conductors;
//  * the four radial E edges at every wire node have eps and sigma multiplied
//    by m = ln(dx / r0) / ln(dx / a), r0 = wire_r0_factor * dx being the
//    equivalent radius of a bare conductor edge (default exp(-pi/2) dx);
//  * the four H components circulating around every wire segment, and
//    around the one segment beyond each end, have mu divided by m;
//  * the four H components parallel to the wire around every wire node have
//    mu divided by m.
// The last two rules keep every coupling of a radial edge at its unmodified
// strength: scaling only the radial edges and the circulating H inside the
// wire raises the coupling of a radial edge to its parallel H and to the
// circulating H past an end by 1/sqrt(m), which pushes the scheme past its
// stability limit at 0.99 of the Courant step.  All changes are material
// changes, so the discrete energy identity of the Yee scheme still holds.
// A perfect-conductor edge ignores any modification; a component next to two
// wires keeps the factor of the first wire added.  In Debye media the radial
// edges scale the whole permittivity function by m (eps_inf, sigma and each
// pole's increment), a reading of the paper's note that the wire models are
// adapted to Debye media (parity unpinned: the adaptation it cites is not
// available).
void scale_mu(orc_sim* s, int a, const int p[3], double m) {
  A3& h = s->mu[a];
  if (!h.in(p[0], p[1], p[2])) return;
  const size_t li = ((size_t)p[2] * h.n1 + p[1]) * h.n0 + p[0];
  if (s->hmod[a][li]) return;
  s->hmod[a][li] = 1;
  h.v[li] /= m;
}

void apply_wires(orc_sim* s) {
  for (const Wire& w : s->wires) {
    const int u = w.axis, v = (u + 1) % 3, x = (u + 2) % 3;
    const double m = std::log(1.0 / s->P.wire_r0_factor) / std::log(s->dx / w.radius);
    for (int t = 0; t < w.n; ++t) {  // axial edges
      int p[3] = {w.p[0], w.p[1], w.p[2]};
      p[u] += t;
      if (s->E[u].in(p[0], p[1], p[2]))
        s->pec[u][((size_t)p[2] * s->E[u].n1 + p[1]) * s->E[u].n0 + p[0]] = 1;
    }
    for (int t = 0; t <= w.n; ++t) {  // radial edges at every wire node
      for (int d = -1; d <= 0; ++d) {
        const int ax[2] = {v, x};
        for (int r = 0; r < 2; ++r) {
          const int a = ax[r];
          int p[3] = {w.p[0], w.p[1], w.p[2]};
          p[u] += t;
          p[a] += d;
          A3& e = s->eps[a];
          if (!e.in(p[0], p[1], p[2])) continue;
          const size_t li = ((size_t)p[2] * e.n1 + p[1]) * e.n0 + p[0];
          if (s->emod[a][li]) continue;
          s->emod[a][li] = 1;
          s->eps[a].v[li] *= m;
          s->sig[a].v[li] *= m;
          for (int dd = 0; dd < s->npole; ++dd) s->deps[a][dd].v[li] *= m;
        }
      }
    }
    for (int t = -1; t <= w.n; ++t) {  // circulating H, segments s0-1 .. s1
      // H_v sits at v = wire, x = wire +- 1/2; H_x at x = wire, v = wire +- 1/2.
      for (int d = -1; d <= 0; ++d) {
        int p[3] = {w.p[0], w.p[1], w.p[2]};
        p[u] += t;
        p[x] += d;
        scale_mu(s, v, p, m);
        int q[3] = {w.p[0], w.p[1], w.p[2]};
        q[u] += t;
        q[v] += d;
        scale_mu(s, x, q, m);
      }
    }
    for (int t = 0; t <= w.n; ++t)  // parallel H around every node
      for (int dv = -1; dv <= 0; ++dv)
        for (int dx = -1; dx <= 0; ++dx) {
          int p[3] = {w.p[0], w.p[1], w.p[2]};
          p[u] += t;
          p[v] += dv;
          p[x] += dx;
          scale_mu(s, u, p, m);
        }
  }
}

// Lumped elements (Section 2.1, lumped circuit elements): a resistor R or a
// capacitor C across one E edge of length dx in a cell of cross-section dx^2
// is the conductivity dx / (R dx^2) = 1 / (R dx) or the permittivity
// C dx / dx^2 = C / dx, added to the edge's own after the wire changes.
void apply_lumped(orc_sim* s) {
  for (const Lumped& l : s->lumped) {
    A3& target = l.kind == ORC_LUMPED_R ? s->sig[l.axis] : s->eps[l.axis];
    target(l.p[0], l.p[1], l.p[2]) += l.kind == ORC_LUMPED_R ? 1.0 / (l.value * s->dx) : l.value / s->dx;
  }
}

// Lossy coefficients for E = Ca E + Cb curl H.  Literal eq. 4:
// Ca = 1 - sigma dt / eps, Cb = dt / eps.  Semi-implicit (sigma E taken at
// n + 1/2 as the mean of n and n + 1, the modification the paper points to
// for better accuracy): Ca = (1 - x) / (1 + x), Cb = (dt / eps) / (1 + x),
// x = sigma dt / (2 eps).  H: Db = dt / mu (eq. 5).
//
// Debye media (Section 2.4: auxiliary differential equation).  Each pole p
// adds a polarisation current with tau_p dJ_p/dt + J_p = eps0 de_p dE/dt.
// Taken at n + 1/2 with the trapezoidal rule, like sigma E:
//   J_p^{n+1} = k_p J_p^n + beta_p (E^{n+1} - E^n),
//   k_p = (2 tau_p - dt) / (2 tau_p + dt),  beta_p = 2 eps0 de_p / (2 tau_p + dt),
// and Ampere's law eps dE/dt + sigma E + sum_p J_p = curl H (eps = eps0
// eps_inf) at n + 1/2 with J_p as the mean of n and n + 1 gives
//   E^{n+1} = Ca E^n + Cb curl H - sum_p gam_p J_p^n,  gam_p = Cb (1 + k_p) / 2,
//   Ca = (1 - x + y) / (1 + x + y),  Cb = (dt / eps) / (1 + x + y),
// y = sum_p beta_p dt / (2 eps).  With no pole increments y = 0 and the
// semi-implicit lossy coefficients come out unchanged.
int build_coefficients(orc_sim* s) {
  const double dt = s->dt;
  for (int d = 0; d < s->npole; ++d) s->kp[d] = (2.0 * s->tau[d] - dt) / (2.0 * s->tau[d] + dt);
  for (int a = 0; a < 3; ++a) {
    const A3& e = s->eps[a];
    s->Ca[a].init(e.n0, e.n1, e.n2, 0.0);
    s->Cb[a].init(e.n0, e.n1, e.n2, 0.0);
    for (int d = 0; d < s->npole; ++d) {
      s->Jbeta[a][d].init(e.n0, e.n1, e.n2, 0.0);
      s->Jgam[a][d].init(e.n0, e.n1, e.n2, 0.0);
    }
    for (size_t li = 0; li < e.v.size(); ++li) {
      const double ep = s->eps[a].v[li], sg = s->sig[a].v[li];
      if (s->P.loss_mode == ORC_LOSS_EXPLICIT) {
        if (sg * dt / ep >= 2.0) return fail(s, ORC_EUNSTABLE, "explicit loss factor below -1");
        s->Ca[a].v[li] = 1.0 - sg * dt / ep;
        s->Cb[a].v[li] = dt / ep;
      } else {
        const double x = sg * dt / (2.0 * ep);
        double bsum = 0;
        for (int d = 0; d < s->npole; ++d) {
          s->Jbeta[a][d].v[li] = 2.0 * s->deps[a][d].v[li] / (2.0 * s->tau[d] + dt);
          bsum += s->Jbeta[a][d].v[li];
        }
        const double y = bsum * dt / (2.0 * ep);
        s->Ca[a].v[li] = (1.0 - x + y) / (1.0 + x + y);
        s->Cb[a].v[li] = (dt / ep) / (1.0 + x + y);
        for (int d = 0; d < s->npole; ++d) s->Jgam[a][d].v[li] = s->Cb[a].v[li] * (1.0 + s->kp[d]) / 2.0;
      }
    }
    const A3& m = s->mu[a];
    s->Db[a].init(m.n0, m.n1, m.n2, 0.0);
    for (size_t li = 0; li < m.v.size(); ++li) s->Db[a].v[li] = dt / m.v[li];
  }
  return ORC_OK;
}

// Convolutional PML (Section 2.2; recursive convolution).  Depth rho (cells)
// is measured from the inner face of the layer at the component's own
// position along the axis; s = rho / npml;
//   sigma = sigma_max s^m,  kappa = 1 + (kappa_max - 1) s^m,
//   alpha = alpha_max (1 - s)^m_a,  b = exp(-(sigma / kappa + alpha) dt / eps0),
//   c = sigma (b - 1) / (kappa (sigma + kappa alpha)),
// sigma_max = sigma_factor * 0.8 (m + 1) / (eta0 dx).  Outside the layer
// b = c = 0 and 1/kappa = 1, so psi stays 0 and the term is the plain
// difference.
void profile_at(const orc_sim* s, int n_ax, double pos, double& b, double& c, double& ik) {
  b = 0.0; c = 0.0; ik = 1.0;
  const int np = s->P.npml;
  if (np <= 0) return;
  double rho = 0.0;
  if (pos < np) rho = np - pos;
  if (pos > n_ax - np) rho = pos - (n_ax - np);
  if (rho <= 0.0) return;
  const double sfrac = rho / np;
  const double m = s->P.pml_m;
  const double smax = s->P.pml_sigma_factor * 0.8 * (m + 1.0) / (kEta0 * s->dx);
  const double sg = smax * std::pow(sfrac, m);
  const double ka = 1.0 + (s->P.pml_kappa_max - 1.0) * std::pow(sfrac, m);
  const double al = s->P.pml_alpha_max * std::pow(1.0 - sfrac, s->P.pml_ma);
  b = std::exp(-(sg / ka + al) * s->dt / kEps0);
  c = (sg > 0.0) ? sg * (b - 1.0) / (ka * (sg + ka * al)) : 0.0;
  ik = 1.0 / ka;
}

void build_cpml(orc_sim* s) {
  for (int u = 0; u < 3; ++u) {
    const int n = s->N[u];
    s->be[u].resize(n + 1); s->ce[u].resize(n + 1); s->ike[u].resize(n + 1);
    s->bh[u].resize(n); s->ch[u].resize(n); s->ikh[u].resize(n);
    for (int p = 0; p <= n; ++p) profile_at(s, n, p, s->be[u][p], s->ce[u][p], s->ike[u][p]);
    for (int p = 0; p < n; ++p) profile_at(s, n, p + 0.5, s->bh[u][p], s->ch[u][p], s->ikh[u][p]);
  }
  for (int a = 0; a < 3; ++a)
    for (int u = 0; u < 3; ++u) {
      if (u == a) continue;
      s->psi[a][u].init(s->E[a].n0, s->E[a].n1, s->E[a].n2);
      s->psi[3 + a][u].init(s->H[a].n0, s->H[a].n1, s->H[a].n2);
    }
}

int finalize(orc_sim* s) {
  if (s->npole && !s->owires.empty()) return fail(s, ORC_EINVAL, "oblique wires in a grid with Debye media");
  if (s->finalized) return ORC_OK;
  for (int a = 0; a < 3; ++a) {
    int ext[3];
    e_extent(s, a, ext);
    s->E[a].init(ext[0], ext[1], ext[2]);
    h_extent(s, a, ext);
    s->H[a].init(ext[0], ext[1], ext[2]);
  }
  for (const Source& q : s->srcs)
    for (const Wire& w : s->wires)
      if (w.axis == q.axis) {
        const int u = w.axis;
        bool on = true;
        for (int b = 0; b < 3; ++b)
          if (b != u && q.p[b] != w.p[b]) on = false;
        if (on && q.p[u] >= w.p[u] && q.p[u] < w.p[u] + w.n)
          return fail(s, ORC_ERANGE, "source on a wire (perfect-conductor) edge");
      }
  build_materials(s);
  apply_wires(s);
  for (const Lumped& l : s->lumped) {
    const A3& e = s->E[l.axis];
    if (s->pec[l.axis][((size_t)l.p[2] * e.n1 + l.p[1]) * e.n0 + l.p[0]])
      return fail(s, ORC_ERANGE, "lumped element on a wire (perfect-conductor) edge");
  }
  apply_lumped(s);
  int rc = build_coefficients(s);
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) {  // the update needs only the coefficients
    s->eps[a] = A3(); s->sig[a] = A3(); s->mu[a] = A3();
    for (int d = 0; d < s->npole; ++d) {
      s->deps[a][d] = A3();
      s->J[a][d].init(s->E[a].n0, s->E[a].n1, s->E[a].n2, 0.0);
    }
    if (s->npole) s->Eprev[a].init(s->E[a].n0, s->E[a].n1, s->E[a].n2, 0.0);
    std::vector<char>().swap(s->emod[a]);
    std::vector<char>().swap(s->hmod[a]);
  }
  build_cpml(s);
  for (Probe& pr : s->probes) pr.rec.assign(s->P.max_steps, 0.0);
  s->finalized = true;
  return ORC_OK;
}

// sum_p gam_p J_p^n of E edge li of component a (0 without poles)
double debye_term(const orc_sim* s, int a, size_t li) {
  double t = 0;
  for (int d = 0; d < s->npole; ++d) t += s->Jgam[a][d].v[li] * s->J[a][d].v[li];
  return t;
}

void update_h(orc_sim* s) {
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  const double d = s->dx;
  A3 &Ex = s->E[0], &Ey = s->E[1], &Ez = s->E[2];
  A3 &Hx = s->H[0], &Hy = s->H[1], &Hz = s->H[2];
  // Hx at (i, j+1/2, k+1/2): eq. 5.
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const double dz = (Ey(i, j, k + 1) - Ey(i, j, k)) / d;
        const double dy = (Ez(i, j + 1, k) - Ez(i, j, k)) / d;
        double& pz = s->psi[3][2](i, j, k);
        double& py = s->psi[3][1](i, j, k);
        pz = s->bh[2][k] * pz + s->ch[2][k] * dz;
        py = s->bh[1][j] * py + s->ch[1][j] * dy;
        Hx(i, j, k) += s->Db[0](i, j, k) * ((dz * s->ikh[2][k] + pz) - (dy * s->ikh[1][j] + py));
      }
  // Hy at (i+1/2, j, k+1/2): dHy/dt = (dEz/dx - dEx/dz) / mu.
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const double dxv = (Ez(i + 1, j, k) - Ez(i, j, k)) / d;
        const double dz = (Ex(i, j, k + 1) - Ex(i, j, k)) / d;
        double& px = s->psi[4][0](i, j, k);
        double& pz = s->psi[4][2](i, j, k);
        px = s->bh[0][i] * px + s->ch[0][i] * dxv;
        pz = s->bh[2][k] * pz + s->ch[2][k] * dz;
        Hy(i, j, k) += s->Db[1](i, j, k) * ((dxv * s->ikh[0][i] + px) - (dz * s->ikh[2][k] + pz));
      }
  // Hz at (i+1/2, j+1/2, k): dHz/dt = (dEx/dy - dEy/dx) / mu.
#pragma omp parallel for schedule(static)
  for (int k = 1; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const double dy = (Ex(i, j + 1, k) - Ex(i, j, k)) / d;
        const double dxv = (Ey(i + 1, j, k) - Ey(i, j, k)) / d;
        double& py = s->psi[5][1](i, j, k);
        double& px = s->psi[5][0](i, j, k);
        py = s->bh[1][j] * py + s->ch[1][j] * dy;
        px = s->bh[0][i] * px + s->ch[0][i] * dxv;
        Hz(i, j, k) += s->Db[2](i, j, k) * ((dy * s->ikh[1][j] + py) - (dxv * s->ikh[0][i] + px));
      }
}

void update_e(orc_sim* s) {
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  const double d = s->dx;
  A3 &Ex = s->E[0], &Ey = s->E[1], &Ez = s->E[2];
  A3 &Hx = s->H[0], &Hy = s->H[1], &Hz = s->H[2];
  // Ex at (i+1/2, j, k): eq. 4.
#pragma omp parallel for schedule(static)
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t li = ((size_t)k * Ex.n1 + j) * Ex.n0 + i;
        if (s->pec[0][li]) continue;
        const double dy = (Hz(i, j, k) - Hz(i, j - 1, k)) / d;
        const double dz = (Hy(i, j, k) - Hy(i, j, k - 1)) / d;
        double& py = s->psi[0][1](i, j, k);
        double& pz = s->psi[0][2](i, j, k);
        py = s->be[1][j] * py + s->ce[1][j] * dy;
        pz = s->be[2][k] * pz + s->ce[2][k] * dz;
        Ex(i, j, k) = s->Ca[0](i, j, k) * Ex(i, j, k) +
                      s->Cb[0](i, j, k) * ((dy * s->ike[1][j] + py) - (dz * s->ike[2][k] + pz)) -
                      debye_term(s, 0, li);
      }
  // Ey at (i, j+1/2, k): dEy/dt = ((dHx/dz - dHz/dx) - sigma Ey) / eps.
#pragma omp parallel for schedule(static)
  for (int k = 1; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const size_t li = ((size_t)k * Ey.n1 + j) * Ey.n0 + i;
        if (s->pec[1][li]) continue;
        const double dz = (Hx(i, j, k) - Hx(i, j, k - 1)) / d;
        const double dxv = (Hz(i, j, k) - Hz(i - 1, j, k)) / d;
        double& pz = s->psi[1][2](i, j, k);
        double& px = s->psi[1][0](i, j, k);
        pz = s->be[2][k] * pz + s->ce[2][k] * dz;
        px = s->be[0][i] * px + s->ce[0][i] * dxv;
        Ey(i, j, k) = s->Ca[1](i, j, k) * Ey(i, j, k) +
                      s->Cb[1](i, j, k) * ((dz * s->ike[2][k] + pz) - (dxv * s->ike[0][i] + px)) -
                      debye_term(s, 1, li);
      }
  // Ez at (i, j, k+1/2): dEz/dt = ((dHy/dx - dHx/dy) - sigma Ez) / eps.
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const size_t li = ((size_t)k * Ez.n1 + j) * Ez.n0 + i;
        if (s->pec[2][li]) continue;
        const double dxv = (Hy(i, j, k) - Hy(i - 1, j, k)) / d;
        const double dy = (Hx(i, j, k) - Hx(i, j - 1, k)) / d;
        double& px = s->psi[2][0](i, j, k);
        double& py = s->psi[2][1](i, j, k);
        px = s->be[0][i] * px + s->ce[0][i] * dxv;
        py = s->be[1][j] * py + s->ce[1][j] * dy;
        Ez(i, j, k) = s->Ca[2](i, j, k) * Ez(i, j, k) +
                      s->Cb[2](i, j, k) * ((dxv * s->ike[0][i] + px) - (dy * s->ike[1][j] + py)) -
                      debye_term(s, 2, li);
      }
}

// Ideal lumped current source (the J term of eq. 1): after the normal update
// of its edge, E -= Cb * I / (cross-section area), with I sampled at
// (n + 1/2) dt; I > 0 drives current toward +axis.
void inject_sources(orc_sim* s) {
  const double area = s->dx * s->dx;
  for (const Source& q : s->srcs) {
    const double I = (s->step < (long)q.amps.size()) ? q.amps[s->step] : 0.0;
    const int a = q.axis;
    s->E[a](q.p[0], q.p[1], q.p[2]) -= s->Cb[a](q.p[0], q.p[1], q.p[2]) * I / area;
  }
}

// ---- Oblique thin wire (Section 2.3: the arbitrarily located wire model
// the paper takes from the literature; the formulation here is this
// oracle's reading of that model, see the header) ----
//
// Each wire owns a 1D grid along its axis: nodes r_k = A + k dl t
// (k = 0..n) and segments r_k -> r_{k+1}.  Segment k carries the current
// I_k at times n + 1/2; node k carries the charge per unit length q_k at
// integer times.  Telegraph equations with the in-cell inductance and
// capacitance
//   L' dI_k/dt = E_t,k - (q_{k+1} - q_k) / (C' dl)
//   dq_k/dt    = -(I_k - I_{k-1}) / len_k    (I_{-1} = I_n = 0, len_k = dl / 2 at the two ends)
// with L' = mu0 ln(r0/a) / (2 pi), C' = 2 pi eps0 / ln(r0/a), r0 = wire_r0_factor dx.
//
// Coupling to the grid conserves charge.  The grid holds the wire's charge
// Q_k = q_k len_k at the grid nodes with the trilinear (cloud-in-cell)
// weights S_p(r_k) of r_k.  A current I_k on segment k moves charge from
// r_k to r_{k+1}, so it must enter the grid as edge currents I_k D_k(e)
// whose discrete divergence is -(S(r_{k+1}) - S(r_k)): then Gauss's law on
// the grid tracks the wire's charge exactly, and a steady current leaves
// no charge behind on the grid.  D_k is the density decomposition of
// Esirkepov (Comput. Phys. Commun. 135, 2001) for that displacement, which
// splits the change of a product of 1D shapes into one flux per axis:
//   W_x(i, j, k) = dS_x(i) [S0_y S0_z + dS_y S0_z / 2 + S0_y dS_z / 2 + dS_y dS_z / 3](j, k),
//   D_x(edge i+1/2, j, k) = -sum_{i' <= i} W_x(i', j, k),
// with S0, S1 the 1D tent weights of r_k and r_{k+1} along each axis and
// dS = S1 - S0 (likewise for y and z).  D is dimensionless (edge lengths per
// unit length of displacement in cells): the current density on edge e is
// I_k D_k(e) / dx^2, and the field the segment sees is the adjoint sum
//   E_t,k = sum_e D_k(e) E_e / dl_cells,
// so the wire and the grid exchange energy without loss or gain.  In a
// uniform field E_t,k = t . E exactly (the first moment of D is the
// displacement dl t).  Perfectly conducting edges take no current.
struct OwEntry { int a, p[3]; double d; };

static void owire_pattern(const OWire& w, int k, std::vector<OwEntry>& out) {
  out.clear();
  double r0[3], r1[3];
  for (int u = 0; u < 3; ++u) {
    r0[u] = w.A[u] + k * w.dl * w.t[u];
    r1[u] = w.A[u] + (k + 1) * w.dl * w.t[u];
  }
  // 1D tent weights on the nodes lo[u] .. lo[u] + n[u] - 1 (at most 4, since dl < 2)
  int lo[3], n[3];
  double s0[3][4], ds[3][4];
  for (int u = 0; u < 3; ++u) {
    lo[u] = (int)std::floor(std::min(r0[u], r1[u]));
    n[u] = (int)std::floor(std::max(r0[u], r1[u])) + 2 - lo[u];
    for (int m = 0; m < n[u]; ++m) {
      const double x = lo[u] + m;
      const double a0 = std::max(0.0, 1.0 - std::fabs(r0[u] - x));
      const double a1 = std::max(0.0, 1.0 - std::fabs(r1[u] - x));
      s0[u][m] = a0;
      ds[u][m] = a1 - a0;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    for (int mc = 0; mc < n[c]; ++mc)
      for (int mb = 0; mb < n[b]; ++mb) {
        const double T = s0[b][mb] * s0[c][mc] + 0.5 * ds[b][mb] * s0[c][mc] + 0.5 * s0[b][mb] * ds[c][mc] +
                         ds[b][mb] * ds[c][mc] / 3.0;
        double D = 0.0;
        for (int ma = 0; ma + 1 < n[a]; ++ma) {
          D -= ds[a][ma] * T;
          if (D == 0.0) continue;
          OwEntry e;
          e.a = a;
          e.p[a] = lo[a] + ma;
          e.p[b] = lo[b] + mb;
          e.p[c] = lo[c] + mc;
          e.d = D;
          out.push_back(e);
        }
      }
  }
}

// I^{n+1/2} from E^n and q^n, then q^{n+1} from I^{n+1/2} (before the E update).
//
// Junctions (the multiwire junctions of the oblique-wire model): the end
// nodes of several wires that meet at one point form one node.  Its charge
// Q_J = sum_m q_m len_m (len_m the half segment of member m) changes by the
// currents that flow into the point, and the members share one potential
// V = q_m / C'_m, so q_m = C'_m Q_J / sum_m C'_m len_m.  A wire cut at one of
// its nodes and rejoined there is the uncut wire again.
void owire_currents(orc_sim* s) {
  std::vector<OwEntry> pat;
  for (OWire& w : s->owires) {
    const double dlm = w.dl * s->dx;
    for (int k = 0; k < w.n; ++k) {
      if (k == w.src) {
        w.I[k] = s->step < (long)w.amps.size() ? w.amps[s->step] : 0.0;
        continue;
      }
      owire_pattern(w, k, pat);
      double et = 0.0;
      for (const OwEntry& e : pat) et += e.d * s->E[e.a](e.p[0], e.p[1], e.p[2]);
      et /= w.dl;
      w.I[k] += s->dt / w.Lp * (et - (w.q[k + 1] - w.q[k]) / (w.Cp * dlm));
    }
    if (w.rec >= 0) w.rec_v[s->step] = w.I[w.rec];
  }
  for (OWire& w : s->owires) {
    const double dlm = w.dl * s->dx;
    for (int j = 0; j <= w.n; ++j) {
      if ((j == 0 && w.junc[0] >= 0) || (j == w.n && w.junc[1] >= 0)) continue;
      const double il = j > 0 ? w.I[j - 1] : 0.0, ir = j < w.n ? w.I[j] : 0.0;
      const double len = (j == 0 || j == w.n) ? 0.5 * dlm : dlm;
      w.q[j] -= s->dt * (ir - il) / len;
    }
  }
  for (const OJunction& J : s->ojunc) {
    double Q = 0.0, inflow = 0.0, cap = 0.0;
    for (size_t m = 0; m < J.wire.size(); ++m) {
      const OWire& w = s->owires[J.wire[m]];
      const double len = 0.5 * w.dl * s->dx;
      const int j = J.end[m] ? w.n : 0;
      Q += w.q[j] * len;
      inflow += J.end[m] ? w.I[w.n - 1] : -w.I[0];  // a segment ending at the point brings its current
      cap += w.Cp * len;
    }
    const double V = (Q + s->dt * inflow) / cap;
    for (size_t m = 0; m < J.wire.size(); ++m) {
      OWire& w = s->owires[J.wire[m]];
      w.q[J.end[m] ? w.n : 0] = w.Cp * V;
    }
  }
}

// After the E update and the lumped sources: E -= Cb J with J = I_k D_k / dx^2.
void owire_inject(orc_sim* s) {
  const double area = s->dx * s->dx;
  std::vector<OwEntry> pat;
  for (const OWire& w : s->owires)
    for (int k = 0; k < w.n; ++k) {
      owire_pattern(w, k, pat);
      for (const OwEntry& e : pat) {
        A3& E = s->E[e.a];
        const size_t li = ((size_t)e.p[2] * E.n1 + e.p[1]) * E.n0 + e.p[0];
        if (s->pec[e.a][li]) continue;
        E.v[li] -= s->Cb[e.a].v[li] * w.I[k] * e.d / area;
      }
    }
}

// Debye polarisation currents, after the E update and the sources of the
// step: J_p^{n+1} = k_p J_p^n + beta_p (E^{n+1} - E^n).
void update_j(orc_sim* s) {
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < s->npole; ++d) {
      std::vector<double>& j = s->J[a][d].v;
      const std::vector<double>& b = s->Jbeta[a][d].v;
      const std::vector<double>& e = s->E[a].v;
      const std::vector<double>& e0 = s->Eprev[a].v;
#pragma omp parallel for schedule(static)
      for (size_t li = 0; li < j.size(); ++li) j[li] = s->kp[d] * j[li] + b[li] * (e[li] - e0[li]);
    }
}

// Probe record n: E and line voltage at (n + 1) dt (after the E update of
// step n); loop current at (n + 1/2) dt (the H level of step n).
double probe_value(orc_sim* s, const Probe& pr) {
  const int a = pr.axis;
  if (pr.kind == ORC_PR_E) return s->E[a](pr.p[0], pr.p[1], pr.p[2]);
  if (pr.kind == ORC_PR_VLINE) {
    double v = 0.0;
    for (int t = 0; t < pr.n; ++t) {
      int p[3] = {pr.p[0], pr.p[1], pr.p[2]};
      p[a] += t;
      v += s->E[a](p[0], p[1], p[2]) * s->dx;
    }
    return v;
  }
  // Loop integral of H around the edge, right-hand rule about +axis:
  // I = (H_w(p) - H_w(p - e_v)) dv - (H_v(p) - H_v(p - e_w)) dw.
  const int v = (a + 1) % 3, w = (a + 2) % 3;
  int pv[3] = {pr.p[0], pr.p[1], pr.p[2]};
  pv[v] -= 1;
  int pw[3] = {pr.p[0], pr.p[1], pr.p[2]};
  pw[w] -= 1;
  return (s->H[w](pr.p[0], pr.p[1], pr.p[2]) - s->H[w](pv[0], pv[1], pv[2])) * s->dx -
         (s->H[v](pr.p[0], pr.p[1], pr.p[2]) - s->H[v](pw[0], pw[1], pw[2])) * s->dx;
}

}  // namespace

extern "C" {

int orc_create(const orc_params* p, orc_sim** out) {
  if (!p || !out) return ORC_EINVAL;
  *out = nullptr;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2 || !(p->dx > 0) || p->npml < 0 || p->max_steps < 1)
    return ORC_EINVAL;
  if (p->loss_mode != ORC_LOSS_SEMI && p->loss_mode != ORC_LOSS_EXPLICIT) return ORC_EINVAL;
  if (p->npml > 0 && (p->nx <= 2 * p->npml || p->ny <= 2 * p->npml || p->nz <= 2 * p->npml))
    return ORC_EINVAL;
  if (!(p->wire_r0_factor > 0 && p->wire_r0_factor < 1)) return ORC_EINVAL;
  const double dtmax = p->dx / (kC0 * std::sqrt(3.0));
  const double dt = (p->dt > 0) ? p->dt : 0.99 * dtmax;
  if (dt > dtmax) return ORC_EUNSTABLE;
  orc_sim* s = new orc_sim;
  s->P = *p;
  s->dx = p->dx;
  s->dt = dt;
  s->N[0] = p->nx; s->N[1] = p->ny; s->N[2] = p->nz;
  const size_t nc = (size_t)p->nx * p->ny * p->nz;
  s->c_eps.assign(nc, kEps0);
  s->c_sig.assign(nc, 0.0);
  s->c_mu.assign(nc, kMu0);
  *out = s;
  return ORC_OK;
}

void orc_destroy(orc_sim* s) { delete s; }

int orc_set_threads(int n) {
  if (n < 1) return ORC_EINVAL;
  omp_set_num_threads(n);
  return ORC_OK;
}

double orc_dt(const orc_sim* s) { return s ? s->dt : 0.0; }
const char* orc_last_error(const orc_sim* s) { return s ? s->err.c_str() : "null handle"; }

int orc_set_materials(orc_sim* s, const uint8_t* cm, const orc_material* tab, int n_mat) {
  if (!s || !cm || !tab || n_mat < 1 || n_mat > 256) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  for (int m = 0; m < n_mat; ++m)
    if (!(tab[m].eps_r > 0) || !(tab[m].mu_r > 0) || !(tab[m].sigma >= 0))
      return fail(s, ORC_EINVAL, "bad material");
  const size_t nc = s->c_eps.size();
  for (size_t c = 0; c < nc; ++c) {
    if (cm[c] >= n_mat) return fail(s, ORC_ERANGE, "material id out of table");
    const orc_material& m = tab[cm[c]];
    s->c_eps[c] = m.eps_r * kEps0;
    s->c_sig[c] = m.sigma;
    s->c_mu[c] = m.mu_r * kMu0;
  }
  s->c_mat.assign(cm, cm + nc);
  s->n_mat = n_mat;
  return ORC_OK;
}

int orc_set_debye(orc_sim* s, int n_poles, const double* tau, const double* d_eps) {
  if (!s || !tau || !d_eps || n_poles < 1 || n_poles > 4) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  if (s->n_mat < 1) return fail(s, ORC_ESTATE, "Debye poles before the materials");
  const int n_mat = s->n_mat;
  const uint8_t* cm = s->c_mat.data();
  if (s->P.loss_mode != ORC_LOSS_SEMI) return fail(s, ORC_EINVAL, "Debye media need the semi-implicit loss form");
  for (int d = 0; d < n_poles; ++d)
    if (!(tau[d] > 0) || !std::isfinite(tau[d])) return fail(s, ORC_EINVAL, "bad pole time constant");
  for (int m = 0; m < n_mat * n_poles; ++m)
    if (!(d_eps[m] >= 0) || !std::isfinite(d_eps[m])) return fail(s, ORC_EINVAL, "bad pole increment");
  const size_t nc = s->c_eps.size();
  std::vector<double> cd(nc * n_poles);
  for (size_t c = 0; c < nc; ++c) {
    if (cm[c] >= n_mat) return fail(s, ORC_ERANGE, "material id out of table");
    for (int d = 0; d < n_poles; ++d) cd[c * n_poles + d] = kEps0 * d_eps[cm[c] * n_poles + d];
  }
  s->npole = n_poles;
  for (int d = 0; d < n_poles; ++d) s->tau[d] = tau[d];
  s->c_deps.swap(cd);
  return ORC_OK;
}

int orc_add_wire(orc_sim* s, int axis, int i, int j, int k, int n, double radius) {
  if (!s || axis < 0 || axis > 2 || n < 1) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  if (!(radius > 0) || !(radius < 0.5 * s->dx)) return fail(s, ORC_EINVAL, "radius out of (0, dx/2)");
  const int p[3] = {i, j, k};
  for (int b = 0; b < 3; ++b) {
    const int hi = s->N[b];
    if (p[b] < 0 || p[b] > hi) return fail(s, ORC_ERANGE, "wire node outside the grid");
  }
  if (p[axis] + n > s->N[axis]) return fail(s, ORC_ERANGE, "wire leaves the grid");
  Wire w{axis, {i, j, k}, n, radius};
  s->wires.push_back(w);
  return ORC_OK;
}

int orc_add_lumped(orc_sim* s, int kind, int axis, int i, int j, int k, double value) {
  if (!s || axis < 0 || axis > 2 || (kind != ORC_LUMPED_R && kind != ORC_LUMPED_C)) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  if (!(value > 0) || !std::isfinite(value)) return fail(s, ORC_EINVAL, "lumped value not positive");
  const int p[3] = {i, j, k};
  if (!e_interior(s, axis, p)) return fail(s, ORC_ERANGE, "lumped edge outside the updated edges");
  s->lumped.push_back({kind, axis, {i, j, k}, value});
  return ORC_OK;
}

// Non-ideal sources as their Norton equivalents: a current source I with a
// shunt resistance r (r <= 0: ideal), or a voltage source V with a series
// resistance r > 0, which is the current V / r in parallel with r.  Positive
// values drive current toward +axis inside the source (the +axis end is the
// positive terminal of a voltage source).
int orc_add_source_r(orc_sim* s, int kind, int axis, int i, int j, int k, const double* amps, int n, double r) {
  if (!s || !amps || n < 1 || (kind != ORC_SRC_CURRENT && kind != ORC_SRC_VOLTAGE)) return ORC_EINVAL;
  if (kind == ORC_SRC_VOLTAGE && !(r > 0)) return fail(s, ORC_EINVAL, "a voltage source needs r > 0");
  if (!std::isfinite(r)) return fail(s, ORC_EINVAL, "non-finite internal resistance");
  std::vector<double> cur(amps, amps + n);
  if (kind == ORC_SRC_VOLTAGE)
    for (double& v : cur) v /= r;
  int rc = orc_add_source(s, axis, i, j, k, cur.data(), n);
  if (rc || !(r > 0)) return rc;
  return orc_add_lumped(s, ORC_LUMPED_R, axis, i, j, k, r);
}

int orc_add_source(orc_sim* s, int axis, int i, int j, int k, const double* amps, int n) {
  if (!s || axis < 0 || axis > 2 || !amps || n < 1) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  const int p[3] = {i, j, k};
  if (!e_interior(s, axis, p)) return fail(s, ORC_ERANGE, "source edge outside the updated edges");
  for (int t = 0; t < n; ++t)
    if (!std::isfinite(amps[t])) return fail(s, ORC_EINVAL, "non-finite source sample");
  Source q{axis, {i, j, k}, std::vector<double>(amps, amps + n)};
  s->srcs.push_back(q);
  return ORC_OK;
}

int orc_add_probe(orc_sim* s, int kind, int axis, int i, int j, int k, int n, int* id) {
  if (!s || axis < 0 || axis > 2 || kind < 0 || kind > 2 || n < 1) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "setup after finalize");
  const int p[3] = {i, j, k};
  for (int b = 0; b < 3; ++b)
    if (p[b] < 0 || p[b] >= s->N[b]) return fail(s, ORC_ERANGE, "probe node outside the grid");
  if (kind == ORC_PR_VLINE && p[axis] + n > s->N[axis]) return fail(s, ORC_ERANGE, "line leaves the grid");
  if (kind != ORC_PR_VLINE && n != 1) return ORC_EINVAL;
  if (kind == ORC_PR_ILOOP) {
    const int v = (axis + 1) % 3, w = (axis + 2) % 3;
    if (p[v] < 1 || p[w] < 1) return fail(s, ORC_ERANGE, "loop touches a wall");
  }
  Probe pr{kind, axis, {i, j, k}, n, {}};
  s->probes.push_back(pr);
  if (id) *id = (int)s->probes.size() - 1;
  return ORC_OK;
}

int orc_add_oblique_wire(orc_sim* s, const double* a, const double* b, double radius, int src_seg,
                         const double* amps, int n_amps, int rec_seg, int* id) {
  if (!s || !a || !b || n_amps < 0 || (n_amps > 0 && !amps)) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "grid already stepped");
  double d[3], len2 = 0.0;
  for (int u = 0; u < 3; ++u) {
    if (!std::isfinite(a[u]) || !std::isfinite(b[u])) return fail(s, ORC_EINVAL, "end point not finite");
    const double lo = s->P.npml + 1.0, hi = s->N[u] - s->P.npml - 2.0;
    if (a[u] < lo || a[u] > hi || b[u] < lo || b[u] > hi) return fail(s, ORC_ERANGE, "wire reaches the CPML or the wall");
    d[u] = b[u] - a[u];
    len2 += d[u] * d[u];
  }
  const double len = std::sqrt(len2);
  if (!(len >= 1.0)) return fail(s, ORC_EINVAL, "wire shorter than one cell");
  const double r0 = s->P.wire_r0_factor * s->dx;
  if (!(radius > 0) || !(radius < r0)) return fail(s, ORC_EINVAL, "radius out of (0, r0)");
  OWire w;
  w.n = (int)std::floor(len);
  w.dl = len / w.n;
  for (int u = 0; u < 3; ++u) { w.A[u] = a[u]; w.t[u] = d[u] / len; }
  if (src_seg < -1 || src_seg >= w.n || rec_seg < -1 || rec_seg >= w.n) return fail(s, ORC_ERANGE, "segment index");
  const double lg = std::log(r0 / radius);
  w.Lp = kMu0 * lg / (2.0 * kPi);
  w.Cp = 2.0 * kPi * kEps0 / lg;
  w.src = src_seg;
  w.rec = rec_seg;
  w.amps.assign(amps, amps + n_amps);
  w.I.assign(w.n, 0.0);
  w.q.assign(w.n + 1, 0.0);
  w.rec_v.assign(rec_seg >= 0 ? s->P.max_steps : 0, 0.0);
  s->owires.push_back(w);
  if (id) *id = (int)s->owires.size() - 1;
  return ORC_OK;
}

int orc_join_oblique_wires(orc_sim* s, int n, const int* ids, const int* ends) {
  if (!s || n < 2 || !ids || !ends) return ORC_EINVAL;
  if (s->finalized) return fail(s, ORC_ESTATE, "grid already stepped");
  OJunction J;
  double p0[3] = {0, 0, 0};
  for (int m = 0; m < n; ++m) {
    if (ids[m] < 0 || ids[m] >= (int)s->owires.size() || (ends[m] != 0 && ends[m] != 1))
      return fail(s, ORC_EINVAL, "bad wire id or end");
    const OWire& w = s->owires[ids[m]];
    if (w.junc[ends[m]] >= 0) return fail(s, ORC_EINVAL, "wire end already in a junction");
    for (int q = 0; q < m; ++q)
      if (ids[q] == ids[m] && ends[q] == ends[m]) return fail(s, ORC_EINVAL, "wire end listed twice");
    double p[3];
    for (int u = 0; u < 3; ++u) p[u] = w.A[u] + (ends[m] ? w.n * w.dl * w.t[u] : 0.0);
    if (m == 0)
      std::memcpy(p0, p, sizeof(p0));
    else
      for (int u = 0; u < 3; ++u)
        if (std::fabs(p[u] - p0[u]) > 1e-6) return fail(s, ORC_EINVAL, "joined wire ends do not meet");
    J.wire.push_back(ids[m]);
    J.end.push_back(ends[m]);
  }
  for (int m = 0; m < n; ++m) s->owires[ids[m]].junc[ends[m]] = (int)s->ojunc.size();
  s->ojunc.push_back(J);
  return ORC_OK;
}

int orc_oblique_wire_read(orc_sim* s, int id, double* cur, double* q, double* rec, int n_rec_max, int* n_seg,
                          int* n_written) {
  if (!s || id < 0 || id >= (int)s->owires.size() || n_rec_max < 0) return ORC_EINVAL;
  const OWire& w = s->owires[id];
  if (n_seg) *n_seg = w.n;
  if (cur) std::memcpy(cur, w.I.data(), sizeof(double) * w.n);
  if (q) std::memcpy(q, w.q.data(), sizeof(double) * (w.n + 1));
  const int n = w.rec >= 0 ? (int)std::min<long>(s->step, n_rec_max) : 0;
  if (rec && n) std::memcpy(rec, w.rec_v.data(), sizeof(double) * n);
  if (n_written) *n_written = n;
  return ORC_OK;
}

int orc_step(orc_sim* s, int n_steps) {
  if (!s || n_steps < 0) return ORC_EINVAL;
  int rc = finalize(s);
  if (rc) return rc;
  if (s->step + n_steps > s->P.max_steps) return fail(s, ORC_ERANGE, "beyond max_steps");
  for (int t = 0; t < n_steps; ++t) {
    update_h(s);
    owire_currents(s);
    if (s->npole)
      for (int a = 0; a < 3; ++a) s->Eprev[a].v = s->E[a].v;
    update_e(s);
    inject_sources(s);
    owire_inject(s);
    if (s->npole) update_j(s);
    for (Probe& pr : s->probes) pr.rec[s->step] = probe_value(s, pr);
    ++s->step;
  }
  return ORC_OK;
}

int orc_probe(orc_sim* s, int id, double* out, int n_max, int* n_written) {
  if (!s || !out || id < 0 || id >= (int)s->probes.size()) return ORC_EINVAL;
  int rc = finalize(s);
  if (rc) return rc;
  const int n = (int)std::min<long>(s->step, n_max);
  std::memcpy(out, s->probes[id].rec.data(), sizeof(double) * n);
  if (n_written) *n_written = n;
  return ORC_OK;
}

static A3* comp_array(orc_sim* s, int comp) {
  if (comp < 0 || comp > 5) return nullptr;
  return comp < 3 ? &s->E[comp] : &s->H[comp - 3];
}

int orc_set_field(orc_sim* s, int comp, const double* v) {
  if (!s || !v) return ORC_EINVAL;
  int rc = finalize(s);
  if (rc) return rc;
  A3* f = comp_array(s, comp);
  if (!f) return ORC_EINVAL;
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double x = v[((size_t)k * ny + j) * nx + i];
        if (comp < 3) {
          const int p[3] = {i, j, k};
          const size_t li = ((size_t)k * f->n1 + j) * f->n0 + i;
          if (!e_interior(s, comp, p) || s->pec[comp][li]) x = 0.0;  // perfect conductors
        }
        (*f)(i, j, k) = x;
      }
  return ORC_OK;
}

int orc_get_field(orc_sim* s, int comp, double* v) {
  if (!s || !v) return ORC_EINVAL;
  int rc = finalize(s);
  if (rc) return rc;
  A3* f = comp_array(s, comp);
  if (!f) return ORC_EINVAL;
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) v[((size_t)k * ny + j) * nx + i] = (*f)(i, j, k);
  return ORC_OK;
}

int orc_get_coef(orc_sim* s, int comp, int which, double* v) {
  if (!s || !v || comp < 0 || comp > 5 || which < 0 || which > 1) return ORC_EINVAL;
  if (comp >= 3 && which == 1) return ORC_EINVAL;
  int rc = finalize(s);
  if (rc) return rc;
  A3* f = comp < 3 ? (which == 0 ? &s->Ca[comp] : &s->Cb[comp]) : &s->Db[comp - 3];
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double x = (*f)(i, j, k);
        if (comp < 3) {
          const int p[3] = {i, j, k};
          const size_t li = ((size_t)k * f->n1 + j) * f->n0 + i;
          if (!e_interior(s, comp, p) || s->pec[comp][li]) x = 0.0;
        }
        v[((size_t)k * ny + j) * nx + i] = x;
      }
  return ORC_OK;
}

}  // extern "C"
