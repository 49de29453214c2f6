// fdtd_host.cpp -- host runtime of the MI355X FDTD library: validation, the
// coefficient-class tables, CPML profiles, source and probe tables, the
// workspace layout and the step loop.  Everything here runs on the host;
// device work is issued on the context's stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_dev.h"

using namespace mi355fdtd;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;               // speed of light [m/s]
constexpr double kMu0 = 4.0e-7 * kPi;             // [H/m]
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);    // [F/m]
const double kEta0 = std::sqrt(kMu0 / kEps0);     // free-space impedance [ohm]

struct WireRec { int axis, p[3], n; double radius; };
struct SrcRec { int axis, p[3]; std::vector<double> amps; };
// oblique thin wire as given: end points in cells, radius, driven and
// recorded segment, driving current
struct OWireRec {
  double a[3], b[3], radius;
  int src, rec;
  int junc[2] = {-1, -1};  // junction of the start (0) and end (1) node, -1: open end
  std::vector<double> amps;
};
struct OJuncRec { std::vector<int> wire, end; };
struct LumpedRec { int kind, axis, p[3]; double value; };
struct ProbeRec { int kind, axis, p[3], n; };

// Per-node modifications made by thin wires.
struct NodeMod {
  uint8_t pec = 0;            // bit a: E_a edge is a wire (perfect conductor)
  uint8_t emod = 0, hmod = 0; // bit a: E_a / H_a parameter already scaled
  double em[3] = {1, 1, 1};   // eps and sigma factor of E_a
  double hm[3] = {1, 1, 1};   // mu divisor of H_a
  double deps[3] = {0, 0, 0}; // lumped capacitance of E_a, as permittivity
  double dsig[3] = {0, 0, 0}; // lumped resistance of E_a, as conductivity
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct fdtd_ctx {
  fdtd_params P{};
  hipStream_t stream = nullptr;
  double dt = 0;
  int N[3] = {0, 0, 0};
  long long ncell = 0;
  std::string err;

  // set-up inputs
  std::vector<uint8_t> cell_mat;
  std::vector<fdtd_material> mats;
  // Debye media: pole time constants shared by the grid, eps0 * increment
  // per material and pole; per class the pole factors (dtab, D_STRIDE values)
  int npole = 0;
  double tau[D_MAXPOLE] = {0, 0, 0, 0};
  std::vector<double> mat_deps;       // [material * npole + p]
  std::vector<double> dtab;           // [ncls][D_STRIDE]
  std::vector<uint8_t> dflag;         // [ncls]
  long long debye_nodes = 0;          // nodes whose class has a pole term
  size_t off_j = 0, off_dtab = 0, off_dflag = 0;
  DebyeView<float> d32 = {};
  DebyeView<double> d64 = {};
  std::vector<WireRec> wires;
  std::vector<SrcRec> srcs;
  std::vector<OWireRec> owr;
  std::vector<OJuncRec> ojn;
  std::vector<int> jn_off, jn_q;
  std::vector<double> jn_a, jn_c;
  size_t off_jn_off = 0, off_jn_q = 0, off_jn_a = 0, off_jn_c = 0;
  std::vector<OWireParam> ow_par;
  std::vector<int> ow_seg_off, ow_eoff, ow_jseg;
  std::vector<long long> ow_gkey, ow_ekey;
  std::vector<double> ow_gw, ow_jw, ow_amp;
  int ow_seg = 0;
  std::vector<int> ow_wsrc, ow_gedge;  // source-list row of each touched edge; edge of each gather term
  size_t off_ow_wsrc = 0, off_ow_gedge = 0, off_ow_e1 = 0;
  size_t off_ow_par = 0, off_ow_segoff = 0, off_ow_gkey = 0, off_ow_gw = 0, off_ow_ekey = 0, off_ow_eoff = 0,
         off_ow_jseg = 0, off_ow_jw = 0, off_ow_amp = 0, off_ow_cur = 0, off_ow_q = 0, off_ow_rec = 0;
  OWireView ow_view{};
  std::vector<LumpedRec> lumped;
  std::vector<ProbeRec> probes;

  // frozen tables (host copies)
  bool frozen = false;
  int ncls = 0;
  int cls16 = 0;
  std::vector<uint16_t> cls_id;       // per node
  std::vector<double> ctab;           // [ncls][K_NCOEF], Cb and Db already / dx
  std::vector<double> prof[3];        // [P_NROW][2 npml]
  std::vector<int> src_comp;
  std::vector<long long> src_idx;
  std::vector<double> src_amp;        // [n_src][max_steps], Cb I / dx^2
  std::vector<int> src_first;         // [nx * ny] first source of each column, -1 if none
  std::vector<int> src_kr;            // [nx * ny] planes of a column's sources, kmin | kmax << 16
  size_t off_src_first = 0, off_src_kr = 0;
  std::vector<int> pr_off, term_comp;
  std::vector<long long> term_idx;
  std::vector<double> term_w;
  size_t ws_bytes = 0;
  // workspace offsets (bytes from the workspace base)
  size_t off_f = 0, off_psi[2][3] = {{0, 0, 0}, {0, 0, 0}}, off_zpl = 0, off_cls = 0, off_ctab = 0, off_prof = 0;
  size_t off_src_comp = 0, off_src_idx = 0, off_amp = 0, off_pr_off = 0, off_term_comp = 0;
  size_t off_term_idx = 0, off_term_w = 0, off_out = 0, psi_elems[3] = {0, 0, 0};
  std::vector<uint8_t> cls8;          // staging for 1-byte class ids
  // fused tile lists of a grid with a CPML (i0, j0, k0, k1 per tile): the
  // interior tiles first, then the CPML tiles; rebuilt when TY or TZ change
  size_t off_tiles = 0, max_tiles = 0;
  std::vector<int> tl;
  // tile counts of the 4 CPML groups, of group 4 (tiles that read an oblique
  // wire's amplitudes) and of its first part, the tiles clear of the x and y
  // slabs (two-step pass only)
  int tl_cnt[6] = {0, 0, 0, 0, 0, 0}, tl_var = -1, tl_ty = -1, tl_kz = -1;
  // the CPML tile groups run on a second stream, concurrently with the
  // clear tiles: fork and join events around each pass
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // third stream for the oblique-wire kernels of a pass over tile lists;
  // ev_src marks their end for the tiles that read their amplitudes
  hipStream_t aux2 = nullptr;
  hipEvent_t ev_src = nullptr;

  // bound state
  char* ws = nullptr;
  int cur = 0;
  long long steps_done = 0;
  int variant = FDTD_KERNEL_AUTO, tile_y = 0, tile_z = 0;
  // graph replay (fdtd_set_graph): G steps captured once per parity of the
  // field set they start from, replayed with the step taken from a device
  // counter at off_dstep
  int graph_steps = 0;
  long long graph_key = -1;          // launch shape the graphs were captured for
  size_t off_dstep = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // kernel timing: a ring of event pairs, drained when a slot is reused
  bool timing = false;
  static constexpr int kRing = 64;
  hipEvent_t ev0[kRing] = {}, ev1[kRing] = {};
  int ev_steps[kRing] = {};          // steps covered by each event pair
  int ev_next = 0, ev_pending = 0;
  double timed_ms = 0;
  long long timed_steps = 0;
  GridView<float> v32[2][2] = {};   // [input set][output set]
  GridView<double> v64[2][2] = {};
};

int fdtd_fail_code(fdtd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

namespace {

int fail(fdtd_ctx* c, int code, const std::string& msg) { return fdtd_fail_code(c, code, msg); }

int tsize(const fdtd_ctx* c) { return c->P.precision == 64 ? 8 : 4; }

long long node_index(const fdtd_ctx* c, int i, int j, int k) {
  return (long long)i + (long long)c->N[0] * ((long long)j + (long long)c->N[1] * k);
}

bool node_in(const fdtd_ctx* c, const int p[3]) {
  for (int b = 0; b < 3; ++b)
    if (p[b] < 0 || p[b] >= c->N[b]) return false;
  return true;
}

// An E edge the update touches: every transverse index in [1, n-1].
bool edge_updated(const fdtd_ctx* c, int a, const int p[3]) {
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      if (p[b] < 0 || p[b] >= c->N[b]) return false;
    } else if (p[b] < 1 || p[b] > c->N[b] - 1) {
      return false;
    }
  }
  return true;
}

// -------------------------------------------------------------------------
// Coefficient classes
// -------------------------------------------------------------------------

// A class: the K_NCOEF coefficients, then the D_STRIDE pole factors.
constexpr int K_ALL = K_NCOEF + D_STRIDE;
using Coefs = std::array<double, K_ALL>;

// Material id of cell (i, j, k), or 0xFF outside the grid.
inline uint8_t cell_id(const fdtd_ctx* c, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= c->N[0] || j >= c->N[1] || k >= c->N[2]) return 0xFF;
  return c->cell_mat.empty() ? 0 : c->cell_mat[node_index(c, i, j, k)];
}

// The 8 cells around node (i, j, k): bit pattern di + 2 dj + 4 dk selects
// cell (i - 1 + di, j - 1 + dj, k - 1 + dk).
inline uint64_t node_key(const fdtd_ctx* c, int i, int j, int k) {
  uint64_t key = 0;
  for (int q = 0; q < 8; ++q) {
    const uint64_t id = cell_id(c, i - 1 + (q & 1), j - 1 + ((q >> 1) & 1), k - 1 + ((q >> 2) & 1));
    key |= id << (8 * q);
  }
  return key;
}

// Coefficients of a node from its 8 surrounding cells and wire changes.
// E_a: eps, sigma = arithmetic mean over the 4 cells sharing the edge (all
// must be inside the grid, else the edge lies on a wall and is held at 0).
// H_a: mu = harmonic mean over the (1 or 2) in-grid cells sharing the face.
int node_coefs(fdtd_ctx* c, uint64_t key, const NodeMod* mod, Coefs& out) {
  const double dt = c->dt, dx = c->P.dx;
  auto cell = [&](int q) -> int { return (int)((key >> (8 * q)) & 0xFF); };
  for (int q = K_NCOEF; q < K_ALL; ++q) out[q] = 0.0;
  for (int a = 0; a < 3; ++a) {
    // cells sharing E_a: index along a fixed at +0 (bit a set), others vary
    double eps = 0, sig = 0, de[D_MAXPOLE] = {0, 0, 0, 0};
    bool wall = false;
    for (int s = 0; s < 4; ++s) {
      int bits[3];
      int t = 0;
      for (int b = 0; b < 3; ++b) bits[b] = (b == a) ? 1 : ((s >> (t++)) & 1);
      const int id = cell(bits[0] | (bits[1] << 1) | (bits[2] << 2));
      if (id == 0xFF) { wall = true; break; }
      eps += c->mats[id].eps_r * kEps0;
      sig += c->mats[id].sigma;
      for (int p = 0; p < c->npole; ++p) de[p] += c->mat_deps[(size_t)id * c->npole + p];
    }
    // The table stores ca - 1, not ca: in a conductor ca is close to 1 and an
    // FP32 ca would keep only a few bits of 1 - ca (the loss per step); the
    // kernels evaluate E + ((ca - 1) E + cb curl), the same update.
    // Debye poles (auxiliary differential equation, trapezoidal in time):
    // J_p' = kp J_p + beta_p (E' - E) with beta_p = 2 eps0 de_p / (2 tau_p + dt)
    // enters Ampere's law as the mean of J_p and J_p', which adds
    // y = sum_p beta_p dt / (2 eps) to the denominator of ca and cb and the
    // term -gam_p J_p, gam_p = cb (1 + kp) / 2, to the update.  y = 0 without
    // poles.
    double cam1 = -1.0, cb = 0;  // perfect conductor: E stays 0
    const bool pec = wall || (mod && (mod->pec >> a) & 1);
    if (!pec) {
      eps *= 0.25;
      sig *= 0.25;
      double beta[D_MAXPOLE] = {0, 0, 0, 0}, bsum = 0;
      for (int p = 0; p < c->npole; ++p) {
        de[p] *= 0.25;
        if (mod) de[p] *= mod->em[a];
        beta[p] = 2.0 * de[p] / (2.0 * c->tau[p] + dt);
        bsum += beta[p];
      }
      if (mod) { eps *= mod->em[a]; sig *= mod->em[a]; }
      if (mod) { eps += mod->deps[a]; sig += mod->dsig[a]; }  // lumped R and C
      if (c->P.loss_mode == FDTD_LOSS_EXPLICIT) {
        if (sig * dt / eps >= 2.0) return fail(c, FDTD_EUNSTABLE, "literal eq. 4 loss factor below -1");
        cam1 = -sig * dt / eps;             // ca = 1 - sigma dt / eps
        cb = dt / eps;
      } else {
        const double x = 0.5 * sig * dt / eps, y = 0.5 * bsum * dt / eps;
        cam1 = -2.0 * x / (1.0 + x + y);     // ca = (1 - x + y) / (1 + x + y)
        cb = (dt / eps) / (1.0 + x + y);
      }
      // (a pole with no increment keeps J = 0: its factors stay 0, so that
      // the class carries no pole term)
      for (int p = 0; p < c->npole; ++p) {
        const double kp = (2.0 * c->tau[p] - dt) / (2.0 * c->tau[p] + dt);
        out[K_NCOEF + a * 2 * D_MAXPOLE + 2 * p] = beta[p];
        out[K_NCOEF + a * 2 * D_MAXPOLE + 2 * p + 1] = beta[p] != 0.0 ? cb * (1.0 + kp) / 2.0 : 0.0;
      }
    }
    out[2 * a] = cam1;
    out[2 * a + 1] = cb / dx;
    // cells sharing H_a: index along a varies, others fixed at +0 (bit set)
    double inv = 0;
    int cnt = 0;
    for (int s = 0; s < 2; ++s) {
      int bits[3];
      for (int b = 0; b < 3; ++b) bits[b] = (b == a) ? s : 1;
      const int id = cell(bits[0] | (bits[1] << 1) | (bits[2] << 2));
      if (id == 0xFF) continue;
      inv += 1.0 / (c->mats[id].mu_r * kMu0);
      ++cnt;
    }
    double mu = cnt ? cnt / inv : kMu0;
    if (mod) mu /= mod->hm[a];
    out[K_DBX + a] = dt / mu / dx;
  }
  return FDTD_OK;
}

// Thin-wire modifications (Section 2.3, assigned-parameter model): axial
// edges become perfect conductors; radial E edges at every node get eps and
// sigma times m; H circulating around every segment and the segment past
// each end, and H parallel to the wire around every node, get mu / m.  The
// first wire to touch a component sets its factor; a perfect conductor
// overrides any factor.
void collect_wire_mods(fdtd_ctx* c, std::unordered_map<long long, NodeMod>& mods) {
  for (const WireRec& w : c->wires) {
    const int u = w.axis, v = (u + 1) % 3, x = (u + 2) % 3;
    const double m = std::log(1.0 / c->P.wire_r0_factor) / std::log(c->P.dx / w.radius);
    auto scale_e = [&](const int q[3], int a) {
      if (!node_in(c, q)) return;
      NodeMod& nm = mods[node_index(c, q[0], q[1], q[2])];
      if ((nm.emod >> a) & 1) return;
      nm.emod |= 1 << a;
      nm.em[a] = m;
    };
    auto scale_h = [&](const int q[3], int a) {
      if (!node_in(c, q)) return;
      NodeMod& nm = mods[node_index(c, q[0], q[1], q[2])];
      if ((nm.hmod >> a) & 1) return;
      nm.hmod |= 1 << a;
      nm.hm[a] = m;
    };
    for (int t = 0; t < w.n; ++t) {
      int q[3] = {w.p[0], w.p[1], w.p[2]};
      q[u] += t;
      if (node_in(c, q)) mods[node_index(c, q[0], q[1], q[2])].pec |= 1 << u;
    }
    for (int t = 0; t <= w.n; ++t)
      for (int d = -1; d <= 0; ++d) {
        int q[3] = {w.p[0], w.p[1], w.p[2]};
        q[u] += t;
        q[v] += d;
        scale_e(q, v);
        int r[3] = {w.p[0], w.p[1], w.p[2]};
        r[u] += t;
        r[x] += d;
        scale_e(r, x);
      }
    for (int t = -1; t <= w.n; ++t)
      for (int d = -1; d <= 0; ++d) {
        int q[3] = {w.p[0], w.p[1], w.p[2]};  // H_v at x = wire +- 1/2
        q[u] += t;
        q[x] += d;
        scale_h(q, v);
        int r[3] = {w.p[0], w.p[1], w.p[2]};  // H_x at v = wire +- 1/2
        r[u] += t;
        r[v] += d;
        scale_h(r, x);
      }
    for (int t = 0; t <= w.n; ++t)
      for (int dv = -1; dv <= 0; ++dv)
        for (int dw = -1; dw <= 0; ++dw) {
          int q[3] = {w.p[0], w.p[1], w.p[2]};
          q[u] += t;
          q[v] += dv;
          q[x] += dw;
          scale_h(q, u);
        }
  }
  // Lumped elements (Section 2.1): R across an edge of length dx and
  // cross-section dx^2 is the conductivity 1 / (R dx); C the permittivity
  // C / dx; both add to the edge's own after the wire changes.
  for (const LumpedRec& l : c->lumped) {
    NodeMod& nm = mods[node_index(c, l.p[0], l.p[1], l.p[2])];
    if (l.kind == FDTD_LUMPED_R) nm.dsig[l.axis] += 1.0 / (l.value * c->P.dx);
    else nm.deps[l.axis] += l.value / c->P.dx;
  }
}

struct TupleKey {
  std::array<uint64_t, K_ALL> b;
  bool operator<(const TupleKey& o) const { return b < o.b; }
};

TupleKey tuple_key(const fdtd_ctx* c, const Coefs& v) {
  TupleKey k;
  for (int q = 0; q < K_ALL; ++q) {
    if (c->P.precision == 64) {
      std::memcpy(&k.b[q], &v[q], 8);
    } else {
      const float f = (float)v[q];
      uint32_t u;
      std::memcpy(&u, &f, 4);
      k.b[q] = u;
    }
  }
  return k;
}

int build_classes(fdtd_ctx* c) {
  std::unordered_map<long long, NodeMod> mods;
  collect_wire_mods(c, mods);
  std::map<TupleKey, int> by_tuple;
  std::unordered_map<uint64_t, int> by_key;
  c->ctab.clear();
  c->dtab.clear();
  c->dflag.clear();
  auto intern = [&](const Coefs& v) -> int {
    const TupleKey k = tuple_key(c, v);
    auto it = by_tuple.find(k);
    if (it != by_tuple.end()) return it->second;
    const int id = (int)by_tuple.size();
    by_tuple.emplace(k, id);
    c->ctab.insert(c->ctab.end(), v.begin(), v.begin() + K_NCOEF);
    if (c->npole) {
      c->dtab.insert(c->dtab.end(), v.begin() + K_NCOEF, v.end());
      bool any = false;
      for (int q = K_NCOEF; q < K_ALL; ++q) any = any || v[q] != 0.0;
      c->dflag.push_back(any ? 1 : 0);
    }
    return id;
  };
  c->cls_id.assign((size_t)c->ncell, 0);
  Coefs v;
  for (int k = 0; k < c->N[2]; ++k)
    for (int j = 0; j < c->N[1]; ++j) {
      uint64_t last = ~0ull;
      int last_id = -1;
      for (int i = 0; i < c->N[0]; ++i) {
        const uint64_t key = node_key(c, i, j, k);
        if (key != last) {
          auto it = by_key.find(key);
          if (it == by_key.end()) {
            int rc = node_coefs(c, key, nullptr, v);
            if (rc) return rc;
            it = by_key.emplace(key, intern(v)).first;
          }
          last = key;
          last_id = it->second;
        }
        c->cls_id[node_index(c, i, j, k)] = (uint16_t)std::min(last_id, 65535);
        if ((int)by_tuple.size() > 65535) return fail(c, FDTD_ECLASS, "more than 65535 classes");
      }
    }
  for (const auto& kv : mods) {
    const long long n = kv.first;
    const int i = (int)(n % c->N[0]);
    const int j = (int)((n / c->N[0]) % c->N[1]);
    const int k = (int)(n / ((long long)c->N[0] * c->N[1]));
    int rc = node_coefs(c, node_key(c, i, j, k), &kv.second, v);
    if (rc) return rc;
    const int id = intern(v);
    if ((int)by_tuple.size() > 65535) return fail(c, FDTD_ECLASS, "more than 65535 classes");
    c->cls_id[n] = (uint16_t)id;
  }
  c->ncls = (int)by_tuple.size();
  c->cls16 = c->ncls > 256 ? 1 : 0;
  c->debye_nodes = 0;
  if (c->npole)
    for (long long n = 0; n < c->ncell; ++n) c->debye_nodes += c->dflag[c->cls_id[n]];
  // a source or lumped element must not sit on a wire edge
  for (const SrcRec& s : c->srcs) {
    auto it = mods.find(node_index(c, s.p[0], s.p[1], s.p[2]));
    if (it != mods.end() && ((it->second.pec >> s.axis) & 1))
      return fail(c, FDTD_ERANGE, "source on a wire (perfect-conductor) edge");
  }
  for (const LumpedRec& l : c->lumped) {
    auto it = mods.find(node_index(c, l.p[0], l.p[1], l.p[2]));
    if (it != mods.end() && ((it->second.pec >> l.axis) & 1))
      return fail(c, FDTD_ERANGE, "lumped element on a wire (perfect-conductor) edge");
  }
  return FDTD_OK;
}

// CPML (Section 2.2, recursive convolution).  For depth rho (cells) from the
// layer's inner face, s = rho / npml: sigma = sigma_max s^m,
// kappa = 1 + (kappa_max - 1) s^m, alpha = alpha_max (1 - s)^m_a,
// b = exp(-(sigma / kappa + alpha) dt / eps0),
// c = sigma (b - 1) / (kappa (sigma + kappa alpha)); outside the layer
// b = c = 0, 1/kappa = 1.  The kernels work on raw differences, so c is used
// as is with psi stored premultiplied by dx.  The table holds b - 1 (from
// expm1) rather than b: near the inner face b is within 1e-4 of 1, and an
// FP32 b would keep only a few bits of 1 - b; the kernels update
// psi += (b - 1) psi + c d, which is the same recursion.
void profile(const fdtd_ctx* c, int n, double pos, double& bm1, double& cc, double& ik) {
  bm1 = -1; cc = 0; ik = 1;
  const int np = c->P.npml;
  double rho = 0;
  if (pos < np) rho = np - pos;
  else if (pos > n - np) rho = pos - (n - np);
  if (rho <= 0) return;
  const double s = rho / np, m = c->P.pml_m;
  const double smax = c->P.pml_sigma_factor * 0.8 * (m + 1.0) / (kEta0 * c->P.dx);
  const double sg = smax * std::pow(s, m);
  const double ka = 1.0 + (c->P.pml_kappa_max - 1.0) * std::pow(s, m);
  const double al = c->P.pml_alpha_max * std::pow(1.0 - s, c->P.pml_ma);
  bm1 = std::expm1(-(sg / ka + al) * c->dt / kEps0);
  cc = sg > 0 ? sg * bm1 / (ka * (sg + ka * al)) : 0.0;
  ik = 1.0 / ka;
}

void build_cpml(fdtd_ctx* c) {
  const int np = c->P.npml;
  for (int u = 0; u < 3; ++u) {
    c->prof[u].assign((size_t)P_NROW * 2 * np, 0.0);
    for (int l = 0; l < 2 * np; ++l) {
      const int pos = l < np ? l : c->N[u] - 2 * np + l;
      double* r = c->prof[u].data();
      profile(c, c->N[u], pos, r[P_BE * 2 * np + l], r[P_CE * 2 * np + l], r[P_IKE * 2 * np + l]);
      profile(c, c->N[u], pos + 0.5, r[P_BH * 2 * np + l], r[P_CH * 2 * np + l], r[P_IKH * 2 * np + l]);
    }
  }
}

void build_sources_probes(fdtd_ctx* c) {
  const int ms = c->P.max_steps;
  c->src_comp.clear(); c->src_idx.clear(); c->src_amp.assign((size_t)c->srcs.size() * ms, 0.0);
  for (size_t s = 0; s < c->srcs.size(); ++s) {
    const SrcRec& r = c->srcs[s];
    const long long n = node_index(c, r.p[0], r.p[1], r.p[2]);
    c->src_comp.push_back(r.axis);
    c->src_idx.push_back(n);
    const double cb = c->ctab[(size_t)c->cls_id[n] * K_NCOEF + 2 * r.axis + 1] * c->P.dx;  // Cb
    const double area = c->P.dx * c->P.dx;
    for (int t = 0; t < ms && t < (int)r.amps.size(); ++t) c->src_amp[s * ms + t] = cb * r.amps[t] / area;
  }
  c->pr_off.assign(1, 0); c->term_comp.clear(); c->term_idx.clear(); c->term_w.clear();
  const double d = c->P.dx;
  auto term = [&](int comp, int i, int j, int k, double w) {
    c->term_comp.push_back(comp);
    c->term_idx.push_back(node_index(c, i, j, k));
    c->term_w.push_back(w);
  };
  for (const ProbeRec& p : c->probes) {
    const int a = p.axis;
    if (p.kind == FDTD_PR_E) {
      term(a, p.p[0], p.p[1], p.p[2], 1.0);
    } else if (p.kind == FDTD_PR_VLINE) {
      for (int t = 0; t < p.n; ++t) {
        int q[3] = {p.p[0], p.p[1], p.p[2]};
        q[a] += t;
        term(a, q[0], q[1], q[2], d);
      }
    } else {  // loop: (H_w(p) - H_w(p - e_v)) dv - (H_v(p) - H_v(p - e_w)) dw
      const int v = (a + 1) % 3, w = (a + 2) % 3;
      int qv[3] = {p.p[0], p.p[1], p.p[2]};
      qv[v] -= 1;
      int qw[3] = {p.p[0], p.p[1], p.p[2]};
      qw[w] -= 1;
      term(3 + w, p.p[0], p.p[1], p.p[2], d);
      term(3 + w, qv[0], qv[1], qv[2], -d);
      term(3 + v, p.p[0], p.p[1], p.p[2], -d);
      term(3 + v, qw[0], qw[1], qw[2], d);
    }
    c->pr_off.push_back((int)c->term_comp.size());
  }
}

int owire_segments(const OWireRec& r) {
  double l2 = 0.0;
  for (int u = 0; u < 3; ++u) l2 += (r.b[u] - r.a[u]) * (r.b[u] - r.a[u]);
  return (int)std::floor(std::sqrt(l2));
}

// Charge-conserving coupling of an oblique wire to the grid (Section 2.3,
// the arbitrarily located wire model; formulation of this library).  The
// grid carries the wire's node charges with the tent (cloud-in-cell)
// weights of the node positions, so a segment current I moving charge from
// node p0 to node p1 must enter the grid as edge currents I D(e) whose
// divergence is minus the change of those weights.  D is taken from
// Esirkepov's density decomposition (2001): with per-axis tent weights
// w0_u, w1_u at the two nodes and dw_u = w1_u - w0_u, the change
// prod w1 - prod w0 splits into one term per axis,
//   X_a = dw_a * (w0_b w0_c + (dw_b w0_c + w0_b dw_c) / 2 + dw_b dw_c / 3),
// and the flux along a through the edge after node i is minus the running
// sum of X_a up to i.  The wire samples the field with the same D (the
// adjoint), so the exchange of energy is exact and a uniform field gives
// E_t = t . E.  Each segment spans less than two cells, so each axis has at
// most four tent nodes.
struct OwTerm { int comp, i, j, k; double d; };

static void owire_flux(const double p0[3], const double p1[3], std::vector<OwTerm>& terms) {
  terms.clear();
  int base[3], cnt[3];
  double w0[3][4] = {}, dw[3][4] = {};
  for (int u = 0; u < 3; ++u) {
    const double lo = std::min(p0[u], p1[u]), hi = std::max(p0[u], p1[u]);
    base[u] = (int)std::floor(lo);
    cnt[u] = (int)std::floor(hi) - base[u] + 2;
    for (int m = 0; m < cnt[u]; ++m) {
      const double node = base[u] + m;
      const double t0 = 1.0 - std::fabs(p0[u] - node), t1 = 1.0 - std::fabs(p1[u] - node);
      w0[u][m] = t0 > 0.0 ? t0 : 0.0;
      dw[u][m] = (t1 > 0.0 ? t1 : 0.0) - w0[u][m];
    }
  }
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, cax = (a + 2) % 3;
    for (int mc = 0; mc < cnt[cax]; ++mc)
      for (int mb = 0; mb < cnt[b]; ++mb) {
        const double tr = w0[b][mb] * w0[cax][mc] + 0.5 * (dw[b][mb] * w0[cax][mc] + w0[b][mb] * dw[cax][mc]) +
                          dw[b][mb] * dw[cax][mc] / 3.0;
        double flux = 0.0;
        for (int ma = 0; ma + 1 < cnt[a]; ++ma) {
          flux -= dw[a][ma] * tr;
          if (flux == 0.0) continue;
          int q[3];
          q[a] = base[a] + ma;
          q[b] = base[b] + mb;
          q[cax] = base[cax] + mc;
          terms.push_back({a, q[0], q[1], q[2], flux});
        }
      }
  }
}

// Tables of every oblique wire: the telegraph factors, per segment its
// gather terms (E key, D / dl), per touched E edge its injection terms
// (segment, D / dx, for E -= (Cb / dx) sum D I / dx) in increasing segment
// order, and the driving current.
void build_owires(fdtd_ctx* c) {
  const int ms = c->P.max_steps;
  const double dx = c->P.dx, r0 = c->P.wire_r0_factor * dx;
  c->ow_par.clear(); c->ow_seg_off.clear(); c->ow_gkey.clear(); c->ow_gw.clear();
  c->ow_ekey.clear(); c->ow_eoff.clear(); c->ow_jseg.clear(); c->ow_jw.clear();
  c->ow_amp.assign(c->owr.size() * (size_t)ms, 0.0);
  struct Inj { long long key; int seg; double w; };
  std::vector<Inj> inj;
  std::vector<OwTerm> terms;
  int seg0 = 0;
  for (size_t w = 0; w < c->owr.size(); ++w) {
    const OWireRec& r = c->owr[w];
    double d[3], len = 0.0;
    for (int u = 0; u < 3; ++u) { d[u] = r.b[u] - r.a[u]; len += d[u] * d[u]; }
    len = std::sqrt(len);
    const int n = owire_segments(r);
    const double dl = len / n, dlm = dl * dx, lg = std::log(r0 / r.radius);
    const double Lp = kMu0 * lg / (2.0 * kPi), Cp = 2.0 * kPi * kEps0 / lg;
    c->ow_par.push_back({seg0, n, r.src, r.rec, c->dt / Lp, 1.0 / (Cp * dlm), c->dt / dlm, 0.0});
    for (int k = 0; k < n; ++k) {
      double p0[3], p1[3];
      for (int u = 0; u < 3; ++u) {
        p0[u] = r.a[u] + k * dl * d[u] / len;
        p1[u] = r.a[u] + (k + 1) * dl * d[u] / len;
      }
      owire_flux(p0, p1, terms);
      c->ow_seg_off.push_back((int)c->ow_gkey.size());
      for (const OwTerm& t : terms) {
        const long long key = ((long long)t.comp << 40) | node_index(c, t.i, t.j, t.k);
        c->ow_gkey.push_back(key);
        c->ow_gw.push_back(t.d / dl);
        inj.push_back({key, seg0 + k, t.d / dx});  // the class table holds Cb / dx
      }
    }
    for (int t = 0; t < ms && t < (int)r.amps.size(); ++t) c->ow_amp[w * ms + t] = r.amps[t];
    seg0 += n;
  }
  c->ow_seg_off.push_back((int)c->ow_gkey.size());
  c->ow_seg = seg0;
  std::stable_sort(inj.begin(), inj.end(), [](const Inj& x, const Inj& y) {
    return x.key != y.key ? x.key < y.key : x.seg < y.seg;
  });
  for (size_t e = 0; e < inj.size(); ++e) {
    if (e == 0 || inj[e].key != inj[e - 1].key) {
      c->ow_ekey.push_back(inj[e].key);
      c->ow_eoff.push_back((int)e);
    }
    c->ow_jseg.push_back(inj[e].seg);
    c->ow_jw.push_back(inj[e].w);
  }
  c->ow_eoff.push_back((int)inj.size());
  c->ow_gedge.clear();  // e_key is sorted, so each gather term finds its edge by bisection
  for (long long key : c->ow_gkey)
    c->ow_gedge.push_back((int)(std::lower_bound(c->ow_ekey.begin(), c->ow_ekey.end(), key) - c->ow_ekey.begin()));
  // junction members: index of the end node in q (wire w's nodes start at
  // seg0 + w), half segment length (m) and C'
  c->jn_off.assign(1, 0);
  c->jn_q.clear(); c->jn_a.clear(); c->jn_c.clear();
  for (const OJuncRec& J : c->ojn) {
    for (size_t m = 0; m < J.wire.size(); ++m) {
      const int w = J.wire[m];
      const OWireRec& r = c->owr[w];
      const OWireParam& p = c->ow_par[w];
      double len = 0.0;
      for (int u = 0; u < 3; ++u) len += (r.b[u] - r.a[u]) * (r.b[u] - r.a[u]);
      const double dlm = std::sqrt(len) / p.nseg * dx, lg = std::log(r0 / r.radius);
      c->jn_q.push_back(p.seg0 + w + (J.end[m] ? p.nseg : 0));
      c->jn_a.push_back(0.5 * dlm);
      c->jn_c.push_back(2.0 * kPi * kEps0 / lg);
    }
    c->jn_off.push_back((int)c->jn_q.size());
  }
}

// The wires' touched edges join the source list after the ideal sources
// (their amplitudes, zero here, are written on the device each step).  The
// list is then grouped by column (stable, so a node keeps its sources in
// the order they were added, the wires' last), and each column records its
// run and planes.  At most 2^20 sources, 2047 in one column (EINVAL).
int group_sources(fdtd_ctx* c) {
  const size_t ms = (size_t)c->P.max_steps, nreg = c->src_comp.size(), ne = c->ow_ekey.size();
  const long long sxy = (long long)c->N[0] * c->N[1];
  for (long long key : c->ow_ekey) {
    c->src_comp.push_back((int)(key >> 40));
    c->src_idx.push_back(key & ((1ll << 40) - 1));
  }
  c->src_amp.resize((nreg + ne) * ms, 0.0);
  const size_t n = c->src_comp.size();
  if (n >= (size_t(1) << 20)) return fail(c, FDTD_EINVAL, "more than 2^20 sources and oblique-wire edges");
  std::vector<int> ord(n);
  for (size_t s = 0; s < n; ++s) ord[s] = (int)s;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return c->src_idx[a] % sxy < c->src_idx[b] % sxy; });
  std::vector<int> comp(n);
  std::vector<long long> idx(n);
  std::vector<double> amp(n * ms);
  c->ow_wsrc.assign(ne, 0);
  for (size_t s = 0; s < n; ++s) {
    const int o = ord[s];
    comp[s] = c->src_comp[o];
    idx[s] = c->src_idx[o];
    std::copy(c->src_amp.begin() + (size_t)o * ms, c->src_amp.begin() + (size_t)(o + 1) * ms,
              amp.begin() + s * ms);
    if ((size_t)o >= nreg) c->ow_wsrc[o - nreg] = (int)s;
  }
  c->src_comp.swap(comp);
  c->src_idx.swap(idx);
  c->src_amp.swap(amp);
  // per column: its run (first | count << 20) and its planes (kmin | kmax
  // << 16, planes beyond 65535 clamped: such a column is always scanned)
  c->src_first.assign((size_t)sxy, -1);
  c->src_kr.assign((size_t)sxy, 0);
  for (size_t s = 0; s < n;) {
    const size_t col = (size_t)(c->src_idx[s] % sxy);
    size_t e = s;
    int lo = 0xffff, hi = 0;
    for (; e < n && (size_t)(c->src_idx[e] % sxy) == col; ++e) {
      const int k = (int)std::min<long long>(c->src_idx[e] / sxy, 0xffff);
      lo = std::min(lo, k);
      hi = std::max(hi, k);
    }
    if (c->N[2] > 0xffff) hi = 0xffff;
    if (e - s >= 2048) return fail(c, FDTD_EINVAL, "more than 2047 sources and oblique-wire edges in one column");
    c->src_first[col] = (int)s | (int)(e - s) << 20;
    c->src_kr[col] = lo | hi << 16;
    s = e;
  }
  return FDTD_OK;
}

void layout(fdtd_ctx* c) {
  const size_t ts = tsize(c);
  const size_t N = (size_t)c->ncell;
  const int np = c->P.npml;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  c->off_f = take(12 * N * ts);
  for (int u = 0; u < 3; ++u) c->psi_elems[u] = 0;
  if (np > 0) {
    c->psi_elems[0] = (size_t)2 * np * c->N[1] * c->N[2];
    c->psi_elems[1] = (size_t)2 * np * c->N[0] * c->N[2];
    c->psi_elems[2] = (size_t)2 * np * c->N[0] * c->N[1];
  }
  for (int s = 0; s < 2; ++s)
    for (int u = 0; u < 3; ++u) c->off_psi[s][u] = take(4 * c->psi_elems[u] * ts);
  c->off_zpl = take((size_t)c->N[0] * c->N[1] * ts);  // zeroed with the fields, never written
  c->off_j = take((size_t)3 * c->npole * N * ts);     // Debye currents, zeroed with the fields
  c->off_cls = take(N * (c->cls16 ? 2 : 1));
  c->off_ctab = take((size_t)c->ncls * K_STRIDE * ts);
  c->off_dtab = take(c->npole ? (size_t)c->ncls * D_STRIDE * ts : 0);
  c->off_dflag = take(c->npole ? (size_t)c->ncls : 0);
  c->off_prof = take(3 * (size_t)P_NROW * 2 * np * ts);
  c->off_src_comp = take(c->src_comp.size() * sizeof(int));
  c->off_src_idx = take(c->src_idx.size() * sizeof(long long));
  c->off_amp = take(c->src_amp.size() * ts);
  c->off_src_first = take(c->src_first.size() * sizeof(int));
  c->off_src_kr = take(c->src_kr.size() * sizeof(int));
  c->off_pr_off = take(c->pr_off.size() * sizeof(int));
  c->off_term_comp = take(c->term_comp.size() * sizeof(int));
  c->off_term_idx = take(c->term_idx.size() * sizeof(long long));
  c->off_term_w = take(c->term_w.size() * sizeof(double));
  c->off_out = take(c->probes.size() * (size_t)c->P.max_steps * sizeof(double));
  c->off_ow_par = take(c->ow_par.size() * sizeof(OWireParam));
  c->off_ow_segoff = take(c->ow_seg_off.size() * sizeof(int));
  c->off_ow_gkey = take(c->ow_gkey.size() * sizeof(long long));
  c->off_ow_gw = take(c->ow_gw.size() * sizeof(double));
  c->off_ow_ekey = take(c->ow_ekey.size() * sizeof(long long));
  c->off_ow_eoff = take(c->ow_eoff.size() * sizeof(int));
  c->off_ow_jseg = take(c->ow_jseg.size() * sizeof(int));
  c->off_ow_jw = take(c->ow_jw.size() * sizeof(double));
  c->off_ow_amp = take(c->ow_amp.size() * sizeof(double));
  c->off_ow_wsrc = take(c->ow_wsrc.size() * sizeof(int));
  c->off_ow_gedge = take(c->ow_gedge.size() * sizeof(int));
  c->off_ow_e1 = take(c->ow_ekey.size() * sizeof(double));
  c->off_jn_off = take(c->jn_off.size() * sizeof(int));
  c->off_jn_q = take(c->jn_q.size() * sizeof(int));
  c->off_jn_a = take(c->jn_a.size() * sizeof(double));
  c->off_jn_c = take(c->jn_c.size() * sizeof(double));
  c->off_ow_cur = take((size_t)c->ow_seg * sizeof(double));
  c->off_ow_q = take((size_t)(c->ow_seg + c->owr.size()) * sizeof(double));
  c->off_ow_rec = take(c->owr.size() * (size_t)c->P.max_steps * sizeof(double));
  c->off_dstep = take(sizeof(int));
  c->max_tiles = 0;
  if (np > 0) {  // bound for 32-wide, 4-high tiles and chunks of >= 4 planes
    c->max_tiles = (size_t)(c->N[0] / 32 + 6) * (c->N[1] / 4 + 6) * (c->N[2] / 4 + 6);
    c->off_tiles = take(c->max_tiles * 4 * sizeof(int));
  }
  // the kernels address every array with 32-bit byte offsets
  bool psi_fits = c->src_amp.size() * ts < (size_t(1) << 32);
  for (int u = 0; u < 3; ++u) psi_fits = psi_fits && 4 * c->psi_elems[u] * ts < (size_t(1) << 32);
  c->ws_bytes = psi_fits ? o : 0;
}

template <typename T>
GridView<T>& view_of(fdtd_ctx* c, int in, int out);
template <>
GridView<float>& view_of<float>(fdtd_ctx* c, int in, int out) { return c->v32[in][out]; }
template <>
GridView<double>& view_of<double>(fdtd_ctx* c, int in, int out) { return c->v64[in][out]; }

template <typename T>
DebyeView<T>& debye_view_of(fdtd_ctx* c);
template <>
DebyeView<float>& debye_view_of<float>(fdtd_ctx* c) { return c->d32; }
template <>
DebyeView<double>& debye_view_of<double>(fdtd_ctx* c) { return c->d64; }

template <typename T>
void fill_view(fdtd_ctx* c, GridView<T>& g, int in, int out) {
  const size_t N = (size_t)c->ncell;
  const int np = c->P.npml;
  char* w = c->ws;
  g.nx = c->N[0]; g.ny = c->N[1]; g.nz = c->N[2]; g.npml = np;
  g.sxy = (long long)c->N[0] * c->N[1];
  g.ncell = c->ncell;
  g.ncls = c->ncls;
  for (int q = 0; q < 6; ++q) {
    g.fi[q] = (const T*)(w + c->off_f) + (size_t)(in * 6 + q) * N;
    g.fo[q] = (T*)(w + c->off_f) + (size_t)(out * 6 + q) * N;
  }
  for (int u = 0; u < 3; ++u) {
    g.pib[u] = np ? (const T*)(w + c->off_psi[in][u]) : nullptr;
    g.pob[u] = np ? (T*)(w + c->off_psi[out][u]) : nullptr;
    g.pel[u] = (unsigned)c->psi_elems[u];
  }
  g.zpl = (const T*)(w + c->off_zpl);
  g.cls = w + c->off_cls;
  g.ctab = (const T*)(w + c->off_ctab);
  for (int u = 0; u < 3; ++u) g.prof[u] = (const T*)(w + c->off_prof) + (size_t)u * P_NROW * 2 * np;
  g.n_src = (int)c->src_comp.size();
  g.max_steps = c->P.max_steps;
  g.src_comp = (const int*)(w + c->off_src_comp);
  g.src_idx = (const long long*)(w + c->off_src_idx);
  g.src_amp = (const T*)(w + c->off_amp);
  g.src_first = (const int*)(w + c->off_src_first);
  g.src_kr = (const int*)(w + c->off_src_kr);
  g.n_probe = (int)c->probes.size();
  g.pr_off = (const int*)(w + c->off_pr_off);
  g.term_comp = (const int*)(w + c->off_term_comp);
  g.term_idx = (const long long*)(w + c->off_term_idx);
  g.term_w = (const double*)(w + c->off_term_w);
  g.pr_out = (double*)(w + c->off_out);
}

template <typename T>
std::vector<T> convert(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

int hip_fail(fdtd_ctx* c, hipError_t e, const char* what) {
  return fail(c, FDTD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
int upload(fdtd_ctx* c) {
  for (int in = 0; in < 2; ++in)
    for (int out = 0; out < 2; ++out) fill_view<T>(c, view_of<T>(c, in, out), in, out);
  const GridView<T>& g = view_of<T>(c, 0, 0);
  hipStream_t st = c->stream;
  // zero fields, CPML state (both sets) and the zero plane
  hipError_t e = hipMemsetAsync(c->ws + c->off_f, 0, c->off_cls - c->off_f, st);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
  const void* cls_src = c->cls_id.data();
  size_t cls_bytes = c->cls_id.size() * 2;
  if (!c->cls16) {
    c->cls8.assign(c->cls_id.begin(), c->cls_id.end());
    cls_src = c->cls8.data();
    cls_bytes = c->cls8.size();
  }
  std::vector<T> tab((size_t)c->ncls * K_STRIDE, T(0)), amp = convert<T>(c->src_amp), prof;
  for (int q = 0; q < c->ncls; ++q)
    for (int t = 0; t < K_NCOEF; ++t) tab[(size_t)q * K_STRIDE + t] = (T)c->ctab[(size_t)q * K_NCOEF + t];
  for (int u = 0; u < 3; ++u)
    for (double x : c->prof[u]) prof.push_back((T)x);
  struct Up { void* dst; const void* src; size_t n; };
  const Up ups[] = {
      {(void*)g.cls, cls_src, cls_bytes},
      {(void*)g.ctab, tab.data(), tab.size() * sizeof(T)},
      {(void*)g.prof[0], prof.data(), prof.size() * sizeof(T)},
      {(void*)g.src_comp, c->src_comp.data(), c->src_comp.size() * sizeof(int)},
      {(void*)g.src_idx, c->src_idx.data(), c->src_idx.size() * sizeof(long long)},
      {(void*)g.src_amp, amp.data(), amp.size() * sizeof(T)},
      {(void*)g.src_first, c->src_first.data(), c->src_first.size() * sizeof(int)},
      {(void*)g.src_kr, c->src_kr.data(), c->src_kr.size() * sizeof(int)},
      {(void*)g.pr_off, c->pr_off.data(), c->pr_off.size() * sizeof(int)},
      {(void*)g.term_comp, c->term_comp.data(), c->term_comp.size() * sizeof(int)},
      {(void*)g.term_idx, c->term_idx.data(), c->term_idx.size() * sizeof(long long)},
      {(void*)g.term_w, c->term_w.data(), c->term_w.size() * sizeof(double)},
  };
  for (const Up& u : ups) {
    if (!u.n) continue;
    e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "upload tables");
  }
  std::vector<T> dt;
  if (c->npole) {
    DebyeView<T>& d = debye_view_of<T>(c);
    d = DebyeView<T>{};
    for (int a = 0; a < 3; ++a)
      for (int p = 0; p < D_MAXPOLE; ++p)  // poles beyond npole alias the last one (read only)
        d.j[a * D_MAXPOLE + p] =
            (T*)(c->ws + c->off_j) + (size_t)(a * c->npole + std::min(p, c->npole - 1)) * (size_t)c->ncell;
    d.dtab = (const T*)(c->ws + c->off_dtab);
    d.dflag = (const unsigned char*)(c->ws + c->off_dflag);
    for (int p = 0; p < c->npole; ++p) d.kp[p] = (T)((2.0 * c->tau[p] - c->dt) / (2.0 * c->tau[p] + c->dt));
    d.npole = c->npole;
    dt = convert<T>(c->dtab);
    e = hipMemcpyAsync((void*)d.dtab, dt.data(), dt.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)d.dflag, c->dflag.data(), c->dflag.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "upload Debye tables");
  }
  e = hipMemsetAsync(g.pr_out, 0, c->probes.size() * (size_t)c->P.max_steps * sizeof(double), st);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
  if (!c->owr.empty()) {
    OWireView& w = c->ow_view;
    w.n_wire = (int)c->owr.size();
    w.max_steps = c->P.max_steps;
    w.n_edge = (int)c->ow_ekey.size();
    w.max_seg = 0;
    for (const OWireParam& q : c->ow_par) w.max_seg = std::max(w.max_seg, q.nseg);
    w.par = (const OWireParam*)(c->ws + c->off_ow_par);
    w.seg_off = (const int*)(c->ws + c->off_ow_segoff);
    w.g_key = (const long long*)(c->ws + c->off_ow_gkey);
    w.g_w = (const double*)(c->ws + c->off_ow_gw);
    w.e_key = (const long long*)(c->ws + c->off_ow_ekey);
    w.e_off = (const int*)(c->ws + c->off_ow_eoff);
    w.j_seg = (const int*)(c->ws + c->off_ow_jseg);
    w.j_w = (const double*)(c->ws + c->off_ow_jw);
    w.amp = (const double*)(c->ws + c->off_ow_amp);
    w.cur = (double*)(c->ws + c->off_ow_cur);
    w.q = (double*)(c->ws + c->off_ow_q);
    w.rec = (double*)(c->ws + c->off_ow_rec);
    w.wsrc = (const int*)(c->ws + c->off_ow_wsrc);
    w.g_edge = (const int*)(c->ws + c->off_ow_gedge);
    w.e1 = (double*)(c->ws + c->off_ow_e1);
    w.n_junc = (int)c->ojn.size();
    w.jn_off = (const int*)(c->ws + c->off_jn_off);
    w.jn_q = (const int*)(c->ws + c->off_jn_q);
    w.jn_a = (const double*)(c->ws + c->off_jn_a);
    w.jn_c = (const double*)(c->ws + c->off_jn_c);
    const Up wups[] = {
        {(void*)w.par, c->ow_par.data(), c->ow_par.size() * sizeof(OWireParam)},
        {(void*)w.seg_off, c->ow_seg_off.data(), c->ow_seg_off.size() * sizeof(int)},
        {(void*)w.g_key, c->ow_gkey.data(), c->ow_gkey.size() * sizeof(long long)},
        {(void*)w.g_w, c->ow_gw.data(), c->ow_gw.size() * sizeof(double)},
        {(void*)w.e_key, c->ow_ekey.data(), c->ow_ekey.size() * sizeof(long long)},
        {(void*)w.e_off, c->ow_eoff.data(), c->ow_eoff.size() * sizeof(int)},
        {(void*)w.j_seg, c->ow_jseg.data(), c->ow_jseg.size() * sizeof(int)},
        {(void*)w.j_w, c->ow_jw.data(), c->ow_jw.size() * sizeof(double)},
        {(void*)w.amp, c->ow_amp.data(), c->ow_amp.size() * sizeof(double)},
        {(void*)w.wsrc, c->ow_wsrc.data(), c->ow_wsrc.size() * sizeof(int)},
        {(void*)w.g_edge, c->ow_gedge.data(), c->ow_gedge.size() * sizeof(int)},
        {(void*)w.jn_off, c->jn_off.data(), c->jn_off.size() * sizeof(int)},
        {(void*)w.jn_q, c->jn_q.data(), c->jn_q.size() * sizeof(int)},
        {(void*)w.jn_a, c->jn_a.data(), c->jn_a.size() * sizeof(double)},
        {(void*)w.jn_c, c->jn_c.data(), c->jn_c.size() * sizeof(double)},
    };
    for (const Up& u : wups) {
      e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail(c, e, "upload oblique-wire tables");
    }
    // currents, charges and the record are contiguous from off_ow_cur
    e = hipMemsetAsync(w.cur, 0, c->off_ow_rec + c->owr.size() * (size_t)c->P.max_steps * sizeof(double) - c->off_ow_cur, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // staging buffers are freed on return
  if (e != hipSuccess) return hip_fail(c, e, "upload");
  return FDTD_OK;
}

int freeze(fdtd_ctx* c) {
  if (c->frozen) return FDTD_OK;
  for (const SrcRec& s : c->srcs)
    if (!edge_updated(c, s.axis, s.p)) return fail(c, FDTD_ERANGE, "source edge on a wall");
  int rc = build_classes(c);
  if (rc) return rc;
  build_cpml(c);
  build_sources_probes(c);
  build_owires(c);
  rc = group_sources(c);
  if (rc) return rc;
  layout(c);
  if (c->ws_bytes == 0) return fail(c, FDTD_EINVAL, "a CPML state array or the source table exceeds 4 GiB");
  c->frozen = true;
  return FDTD_OK;
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

extern "C" {

void fdtd_default_params(fdtd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->pml_m = 3.0;
  p->pml_sigma_factor = 1.0;
  p->pml_kappa_max = 1.0;
  p->pml_alpha_max = 0.0;
  p->pml_ma = 1.0;
  p->loss_mode = FDTD_LOSS_SEMI;
  p->wire_r0_factor = std::exp(-kPi / 2.0);
  p->max_steps = 1;
  p->precision = 32;
}

int fdtd_create(const fdtd_params* p, void* hip_stream, fdtd_ctx** out) {
  if (!p || !out) return FDTD_EINVAL;
  *out = nullptr;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2 || !(p->dx > 0) || !std::isfinite(p->dx)) return FDTD_EINVAL;
  if (p->npml < 0 || (p->npml > 0 && (p->nx <= 2 * p->npml || p->ny <= 2 * p->npml || p->nz <= 2 * p->npml)))
    return FDTD_EINVAL;
  if (p->loss_mode != FDTD_LOSS_SEMI && p->loss_mode != FDTD_LOSS_EXPLICIT) return FDTD_EINVAL;
  if (p->precision != 32 && p->precision != 64) return FDTD_EINVAL;
  if (!(p->wire_r0_factor > 0 && p->wire_r0_factor < 1) || p->max_steps < 1) return FDTD_EINVAL;
  // kernels address each field and CPML array with 32-bit byte offsets
  const long long ts = p->precision == 64 ? 8 : 4;
  if ((long long)p->nx * p->ny * p->nz * ts >= (1ll << 32)) return FDTD_EINVAL;
  if (p->npml > 0 && (!(p->pml_m >= 0) || !(p->pml_kappa_max >= 1) || !(p->pml_alpha_max >= 0) ||
                      !(p->pml_sigma_factor >= 0)))
    return FDTD_EINVAL;
  const double dtmax = p->dx / (kC0 * std::sqrt(3.0));
  const double dt = p->dt > 0 ? p->dt : 0.99 * dtmax;
  if (dt > dtmax) return FDTD_EUNSTABLE;
  fdtd_ctx* c = new fdtd_ctx;
  c->P = *p;
  c->stream = (hipStream_t)hip_stream;
  c->dt = dt;
  c->N[0] = p->nx; c->N[1] = p->ny; c->N[2] = p->nz;
  c->ncell = (long long)p->nx * p->ny * p->nz;
  c->mats.push_back({1.0, 0.0, 1.0});
  *out = c;
  return FDTD_OK;
}

int fdtd_set_materials(fdtd_ctx* c, const uint8_t* cm, const fdtd_material* tab, int n_mat) {
  if (!c || !cm || !tab || n_mat < 1 || n_mat > 255) return fail(c, FDTD_EINVAL, "bad materials arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  for (int m = 0; m < n_mat; ++m) {
    if (!std::isfinite(tab[m].eps_r) || !std::isfinite(tab[m].sigma) || !std::isfinite(tab[m].mu_r))
      return fail(c, FDTD_ENONFINITE, "non-finite material");
    if (!(tab[m].eps_r > 0) || !(tab[m].mu_r > 0) || !(tab[m].sigma >= 0))
      return fail(c, FDTD_EINVAL, "material out of range");
  }
  for (long long n = 0; n < c->ncell; ++n)
    if (cm[n] >= n_mat) return fail(c, FDTD_ERANGE, "material id outside the table");
  c->cell_mat.assign(cm, cm + c->ncell);
  c->mats.assign(tab, tab + n_mat);
  c->npole = 0;  // pole increments refer to a material table: set them again
  c->mat_deps.clear();
  return FDTD_OK;
}

int fdtd_set_debye(fdtd_ctx* c, int n_poles, const double* tau, const double* d_eps) {
  if (!c || !tau || !d_eps || n_poles < 1 || n_poles > D_MAXPOLE) return fail(c, FDTD_EINVAL, "bad Debye arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  if (c->mats.empty()) return fail(c, FDTD_ESTATE, "Debye poles before the materials");
  if (!c->owr.empty()) return fail(c, FDTD_EINVAL, "Debye media in a grid with oblique wires");
  if (c->P.loss_mode != FDTD_LOSS_SEMI) return fail(c, FDTD_EINVAL, "Debye media need the semi-implicit loss form");
  const size_t nm = c->mats.size();
  for (int p = 0; p < n_poles; ++p)
    if (!std::isfinite(tau[p])) return fail(c, FDTD_ENONFINITE, "non-finite pole time constant");
  for (size_t q = 0; q < nm * n_poles; ++q)
    if (!std::isfinite(d_eps[q])) return fail(c, FDTD_ENONFINITE, "non-finite pole increment");
  for (int p = 0; p < n_poles; ++p)
    if (!(tau[p] > 0)) return fail(c, FDTD_EINVAL, "pole time constant not positive");
  for (size_t q = 0; q < nm * n_poles; ++q)
    if (!(d_eps[q] >= 0)) return fail(c, FDTD_EINVAL, "negative pole increment");
  c->npole = n_poles;
  for (int p = 0; p < n_poles; ++p) c->tau[p] = tau[p];
  c->mat_deps.assign(nm * n_poles, 0.0);
  for (size_t q = 0; q < nm * n_poles; ++q) c->mat_deps[q] = kEps0 * d_eps[q];
  return FDTD_OK;
}

int fdtd_add_wire(fdtd_ctx* c, int axis, int i, int j, int k, int n, double radius) {
  if (!c || axis < 0 || axis > 2 || n < 1) return fail(c, FDTD_EINVAL, "bad wire arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  if (!(radius > 0) || !(radius < 0.5 * c->P.dx)) return fail(c, FDTD_EINVAL, "wire radius not in (0, dx/2)");
  const int p[3] = {i, j, k};
  for (int b = 0; b < 3; ++b)
    if (p[b] < 0 || p[b] > c->N[b]) return fail(c, FDTD_ERANGE, "wire node outside the grid");
  if (p[axis] + n > c->N[axis]) return fail(c, FDTD_ERANGE, "wire leaves the grid");
  c->wires.push_back({axis, {i, j, k}, n, radius});
  return FDTD_OK;
}

int fdtd_add_source(fdtd_ctx* c, int kind, int axis, int i, int j, int k, const double* amps, int n) {
  if (!c || kind != FDTD_SRC_CURRENT || axis < 0 || axis > 2 || !amps || n < 1)
    return fail(c, FDTD_EINVAL, "bad source arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  const int p[3] = {i, j, k};
  if (!edge_updated(c, axis, p)) return fail(c, FDTD_ERANGE, "source edge outside the updated edges");
  if (!finite_all(amps, (size_t)n)) return fail(c, FDTD_ENONFINITE, "non-finite source sample");
  c->srcs.push_back({axis, {i, j, k}, std::vector<double>(amps, amps + n)});
  return FDTD_OK;
}

int fdtd_add_oblique_wire(fdtd_ctx* c, const double* a, const double* b, double radius, int src_seg,
                          const double* amps, int n_amps, int rec_seg, int* id) {
  if (!c || !a || !b || n_amps < 0 || (n_amps > 0 && !amps)) return fail(c, FDTD_EINVAL, "bad oblique-wire arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  if (c->npole) return fail(c, FDTD_EINVAL, "oblique wires in a grid with Debye media");
  OWireRec r;
  double l2 = 0.0;
  for (int u = 0; u < 3; ++u) {
    if (!std::isfinite(a[u]) || !std::isfinite(b[u])) return fail(c, FDTD_ENONFINITE, "non-finite wire end point");
    const double lo = c->P.npml + 1.0, hi = c->N[u] - c->P.npml - 2.0;
    if (a[u] < lo || a[u] > hi || b[u] < lo || b[u] > hi)
      return fail(c, FDTD_ERANGE, "oblique wire reaches the CPML or the wall");
    r.a[u] = a[u];
    r.b[u] = b[u];
    l2 += (b[u] - a[u]) * (b[u] - a[u]);
  }
  if (!(std::sqrt(l2) >= 1.0)) return fail(c, FDTD_EINVAL, "oblique wire shorter than one cell");
  if (!(radius > 0) || !(radius < c->P.wire_r0_factor * c->P.dx))
    return fail(c, FDTD_EINVAL, "oblique-wire radius out of (0, wire_r0_factor dx)");
  if (n_amps && !finite_all(amps, (size_t)n_amps)) return fail(c, FDTD_ENONFINITE, "non-finite source sample");
  r.radius = radius;
  const int n = owire_segments(r);
  if (src_seg < -1 || src_seg >= n || rec_seg < -1 || rec_seg >= n) return fail(c, FDTD_ERANGE, "segment index");
  r.src = src_seg;
  r.rec = rec_seg;
  if (n_amps) r.amps.assign(amps, amps + n_amps);
  c->owr.push_back(r);
  if (id) *id = (int)c->owr.size() - 1;
  return FDTD_OK;
}

int fdtd_join_oblique_wires(fdtd_ctx* c, int n, const int* ids, const int* ends) {
  if (!c || n < 2 || !ids || !ends) return fail(c, FDTD_EINVAL, "bad junction arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  OJuncRec J;
  double p0[3] = {0, 0, 0};
  for (int m = 0; m < n; ++m) {
    if (ids[m] < 0 || ids[m] >= (int)c->owr.size() || (ends[m] != 0 && ends[m] != 1))
      return fail(c, FDTD_EINVAL, "bad oblique-wire id or end in a junction");
    const OWireRec& r = c->owr[ids[m]];
    if (r.junc[ends[m]] >= 0) return fail(c, FDTD_EINVAL, "oblique-wire end already in a junction");
    for (int q = 0; q < m; ++q)
      if (ids[q] == ids[m] && ends[q] == ends[m]) return fail(c, FDTD_EINVAL, "oblique-wire end listed twice");
    // the end node as the wire's own segmentation places it
    const int ns = owire_segments(r);
    double d[3], len = 0.0, p[3];
    for (int u = 0; u < 3; ++u) { d[u] = r.b[u] - r.a[u]; len += d[u] * d[u]; }
    len = std::sqrt(len);
    for (int u = 0; u < 3; ++u) p[u] = r.a[u] + (ends[m] ? ns * (len / ns) * d[u] / len : 0.0);
    if (m == 0)
      std::memcpy(p0, p, sizeof(p0));
    else
      for (int u = 0; u < 3; ++u)
        if (std::fabs(p[u] - p0[u]) > 1e-6) return fail(c, FDTD_EINVAL, "joined oblique-wire ends do not meet");
    J.wire.push_back(ids[m]);
    J.end.push_back(ends[m]);
  }
  for (int m = 0; m < n; ++m) c->owr[ids[m]].junc[ends[m]] = (int)c->ojn.size();
  c->ojn.push_back(J);
  return FDTD_OK;
}

int fdtd_oblique_wire_read(fdtd_ctx* c, int id, double* cur, double* q, double* rec, int n_rec_max, int* n_seg,
                           int* n_written) {
  if (!c || id < 0 || id >= (int)c->owr.size() || n_rec_max < 0) return fail(c, FDTD_EINVAL, "bad oblique-wire id");
  const OWireRec& r = c->owr[id];
  const int n = owire_segments(r);
  if (n_seg) *n_seg = n;
  const int nr = r.rec >= 0 ? (int)std::min<long long>((long long)c->steps_done, n_rec_max) : 0;
  if (n_written) *n_written = rec ? nr : 0;
  if (!cur && !q && !(rec && nr)) return FDTD_OK;
  if (!c->ws) return fail(c, FDTD_ESTATE, "no workspace bound");
  hipError_t e = hipStreamSynchronize(c->stream);
  const OWireParam& p = c->ow_par[id];
  if (e == hipSuccess && cur) e = hipMemcpy(cur, c->ow_view.cur + p.seg0, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && q) e = hipMemcpy(q, c->ow_view.q + p.seg0 + id, sizeof(double) * (n + 1), hipMemcpyDeviceToHost);
  if (e == hipSuccess && rec && nr)
    e = hipMemcpy(rec, c->ow_view.rec + (size_t)id * c->P.max_steps, sizeof(double) * nr, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "oblique-wire read");
  return FDTD_OK;
}

int fdtd_add_lumped(fdtd_ctx* c, int kind, int axis, int i, int j, int k, double value) {
  if (!c || (kind != FDTD_LUMPED_R && kind != FDTD_LUMPED_C) || axis < 0 || axis > 2)
    return fail(c, FDTD_EINVAL, "bad lumped-element arguments");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  if (!std::isfinite(value)) return fail(c, FDTD_ENONFINITE, "non-finite lumped value");
  if (!(value > 0)) return fail(c, FDTD_EINVAL, "lumped value not positive");
  const int p[3] = {i, j, k};
  if (!edge_updated(c, axis, p)) return fail(c, FDTD_ERANGE, "lumped edge outside the updated edges");
  c->lumped.push_back({kind, axis, {i, j, k}, value});
  return FDTD_OK;
}

int fdtd_add_source_r(fdtd_ctx* c, int kind, int axis, int i, int j, int k, const double* amps, int n,
                      double r_internal) {
  if (!c || (kind != FDTD_SRC_CURRENT && kind != FDTD_SRC_VOLTAGE) || !amps || n < 1)
    return fail(c, FDTD_EINVAL, "bad source arguments");
  if (!std::isfinite(r_internal)) return fail(c, FDTD_ENONFINITE, "non-finite internal resistance");
  if (kind == FDTD_SRC_VOLTAGE && !(r_internal > 0))
    return fail(c, FDTD_EINVAL, "a voltage source needs a series resistance > 0");
  // Norton equivalent: the current (V / r for a voltage source) in parallel with r
  std::vector<double> cur(amps, amps + n);
  if (kind == FDTD_SRC_VOLTAGE)
    for (double& v : cur) v /= r_internal;
  int rc = fdtd_add_source(c, FDTD_SRC_CURRENT, axis, i, j, k, cur.data(), n);
  if (rc || !(r_internal > 0)) return rc;
  return fdtd_add_lumped(c, FDTD_LUMPED_R, axis, i, j, k, r_internal);
}

int fdtd_add_probe(fdtd_ctx* c, int kind, int axis, int i, int j, int k, int n, int* id) {
  if (!c || kind < 0 || kind > 2 || axis < 0 || axis > 2 || n < 1) return fail(c, FDTD_EINVAL, "bad probe arguments");
  if (kind != FDTD_PR_VLINE && n != 1) return fail(c, FDTD_EINVAL, "only line probes span several cells");
  if (c->frozen) return fail(c, FDTD_ESTATE, "set-up after the workspace size was taken");
  const int p[3] = {i, j, k};
  if (!node_in(c, p)) return fail(c, FDTD_ERANGE, "probe node outside the grid");
  if (kind == FDTD_PR_VLINE && p[axis] + n > c->N[axis]) return fail(c, FDTD_ERANGE, "line leaves the grid");
  if (kind == FDTD_PR_ILOOP && (p[(axis + 1) % 3] < 1 || p[(axis + 2) % 3] < 1))
    return fail(c, FDTD_ERANGE, "loop touches a wall");
  c->probes.push_back({kind, axis, {i, j, k}, n});
  if (id) *id = (int)c->probes.size() - 1;
  return FDTD_OK;
}

int fdtd_finalize(fdtd_ctx* c) {
  if (!c) return FDTD_EINVAL;
  return freeze(c);
}

size_t fdtd_workspace_bytes(fdtd_ctx* c) {
  if (!c) return 0;
  if (freeze(c)) return 0;
  return c->ws_bytes;
}

int fdtd_bind_workspace(fdtd_ctx* c, void* dev, size_t bytes) {
  if (!c) return FDTD_EINVAL;
  int rc = freeze(c);
  if (rc) return rc;
  if (c->ws) return fail(c, FDTD_ESTATE, "workspace already bound");
  if (!dev || bytes < c->ws_bytes) return fail(c, FDTD_ENOMEM, "workspace too small");
  if (((uintptr_t)dev & 255) != 0) return fail(c, FDTD_ENOMEM, "workspace not 256-byte aligned");
  c->ws = (char*)dev;
  rc = c->P.precision == 64 ? upload<double>(c) : upload<float>(c);
  if (rc) c->ws = nullptr;
  return rc;
}

int fdtd_set_kernel(fdtd_ctx* c, int variant, int tile_y, int tile_z) {
  if (!c || variant < FDTD_KERNEL_AUTO || variant > FDTD_KERNEL_TB2 || tile_z < 0 ||
      (tile_y != 0 && tile_y != 4 && tile_y != 8 && tile_y != 12) ||
      (tile_y == 12 && variant != FDTD_KERNEL_TB2))
    return fail(c, FDTD_EINVAL, "bad kernel selection (tile_y in {0, 4, 8}, 12 for the two-step pass; tile_z >= 0)");
  c->variant = variant;
  c->tile_y = tile_y;
  c->tile_z = tile_z;
  return FDTD_OK;
}

}  // extern "C"

namespace {

struct Seg {
  int a, b;
  bool in;
};

// Split [0, n) into the aligned run of `w`-wide pieces that stays clear of
// the CPML (a piece [a, a + w) with a - 1 >= np and a + w <= n - np, a a
// multiple of `align`), and `w_out`-wide pieces for the rest.
std::vector<Seg> segments(int n, int np, int w, int align, int w_out) {
  std::vector<Seg> s;
  int a = (np + 1 + align - 1) / align * align, b = a;
  while (b + w <= n - np) b += w;
  if (b == a) a = b = n;
  for (int x = 0; x < a; x += w_out) s.push_back({x, std::min(x + w_out, a), false});
  for (int x = a; x < b; x += w) s.push_back({x, x + w, true});
  for (int x = b; x < n; x += w_out) s.push_back({x, std::min(x + w_out, n), false});
  return s;
}

// Two-step pieces: [0, n) split into w-wide pieces, those in [a, b) clear
// of the CPML including the h-cell halo (a - h >= np, piece end + h <= n - np);
// a is a multiple of w so that the pieces below it are full width.
// The two-step tiles keep the z CPML table (P_NROW rows of 2 npml values)
// in LDS, room for 2 npml <= 128 values (FP32) or 64 (FP64).
bool tb2_cpml_fits(int npml, int precision) { return 2 * npml <= (precision == 64 ? 64 : 128); }

std::vector<Seg> segments_tb2(int n, int np, int w, int h) {
  std::vector<Seg> s;
  int a = (np + h + w - 1) / w * w, b = a;
  while (b + w <= n - np - h) b += w;
  if (b == a) a = b = n;
  for (int x = 0; x < a; x += w) s.push_back({x, std::min(x + w, a), false});
  for (int x = a; x < b; x += w) s.push_back({x, x + w, true});
  for (int x = b; x < n; x += w) s.push_back({x, std::min(x + w, n), false});
  return s;
}

// z chunk (planes) of the tiles that read an oblique wire's amplitudes.
// They start only once the wire kernels are done, so many short blocks finish
// the pass sooner than a few tall ones: on the lattice-tower scene, one
// plane gave 94.6k Mcell-updates/s, two 93.3k, four 85.8k, eight 74.4k and
// whole chunks 52.2k (the single slanted wire: 101.0k, 101.1k, 99.2k,
// 96.4k, 93.7k).
constexpr int G4_CHUNK = 1;

// Tile lists of the fused and two-step passes for a grid with a CPML (see
// fdtd_ctx::tl and launch_lists_step).
int ensure_tiles(fdtd_ctx* c, int variant, int ty, int kz) {
  if (c->tl_var == variant && c->tl_ty == ty && c->tl_kz == kz) return FDTD_OK;
  const bool tb2 = variant == FDTD_KERNEL_TB2;
  const int np = c->P.npml, nz = c->N[2];
  const std::vector<Seg> xs = tb2 ? segments_tb2(c->N[0], np, 60, 2) : segments(c->N[0], np, 64, 32, 32);
  const std::vector<Seg> ys = tb2 ? segments_tb2(c->N[1], np, ty, 2) : segments(c->N[1], np, ty, ty, ty);
  // z chunks are not split at the slabs: the z CPML branch depends on the
  // plane only, which every thread of a block shares, so the tiles clear of
  // the x and y slabs carry z CPML code at little cost
  // The CPML groups hold few tiles; shorter chunks give their launches
  // enough blocks to fill the device.
  std::vector<Seg> zs[2];
  // Two-step slab groups: at most 20 planes.  On a 512 x 512 x 384 grid,
  // slab chunks of 18-22 planes ran 1-4% faster than 14, 16, 24-30 or 48
  // (measured; the cause is not pinned down).
  const int kzp = tb2 ? std::min(kz, 20) : std::max(8, kz / 4);
  for (int z = 0; z < nz; z += kz) zs[0].push_back({z, std::min(z + kz, nz), true});
  for (int z = 0; z < nz; z += kzp) zs[1].push_back({z, std::min(z + kzp, nz), true});
  std::vector<int> grp[4];
  for (int pass = 0; pass < 2; ++pass)
    for (const Seg& z : zs[pass])
      for (const Seg& y : ys)
        for (const Seg& x : xs) {
          const int q = (x.in ? 0 : 1) | (y.in ? 0 : 2);
          if ((q == 0) != (pass == 0)) continue;
          if (tb2) {
            grp[q].insert(grp[q].end(), {x.a | (x.b - x.a) << 16, y.a | (y.b - y.a) << 16, z.a, z.b});
          } else if (q & 1) {
            for (int xx = x.a; xx < x.b; xx += 32) grp[q].insert(grp[q].end(), {xx, y.a, z.a, z.b});
          } else {
            grp[q].insert(grp[q].end(), {x.a, y.a, z.a, z.b});
          }
        }
  // Group 4: the tiles whose region (halo and pipeline planes included) holds
  // an oblique wire's source edge.  They read the source amplitudes that the
  // wire kernels write before the pass, so they run after those kernels on
  // the second stream (with the all-axes instantiation; fused tiles 32 wide),
  // while the other tiles start at once.
  std::vector<int> grp4, grp4x;  // group 4: from the z-only group, from the others
  if (!c->ow_ekey.empty()) {
    const long long nxl = c->N[0], sxy = nxl * c->N[1];
    std::vector<std::array<int, 3>> pts;
    for (long long key : c->ow_ekey) {
      const long long n = key & ((1ll << 40) - 1);
      pts.push_back({(int)(n % nxl), (int)((n / nxl) % c->N[1]), (int)(n / sxy)});
    }
    for (int q = 0; q < 4; ++q) {
      std::vector<int> keep;
      const int tw = tb2 ? 0 : (q & 1) ? 32 : 64;
      for (size_t t = 0; t < grp[q].size(); t += 4) {
        const int* v = &grp[q][t];
        const int x0 = v[0] & 0xffff, y0 = v[1] & (tb2 ? 0xffff : ~0);
        const int w = tb2 ? v[0] >> 16 : tw, h = tb2 ? v[1] >> 16 : ty;
        bool hit = false;
        for (const auto& p : pts)
          hit = hit || (p[0] >= x0 - 2 && p[0] < x0 + w + 2 && p[1] >= y0 - 2 && p[1] < y0 + h + 2 &&
                        p[2] >= v[2] - 2 && p[2] < v[3] + 2);
        if (!hit) {
          keep.insert(keep.end(), v, v + 4);
          continue;
        }
        // chunks of G4_CHUNK planes (fused tiles 32 wide)
        std::vector<int>& dst = (tb2 && q == 0) ? grp4 : grp4x;
        for (int z = v[2]; z < v[3]; z += G4_CHUNK)
          for (int xx = 0; xx < (tw == 64 ? 2 : 1); ++xx)
            dst.insert(dst.end(), {v[0] + 32 * xx, v[1], z, std::min(z + G4_CHUNK, v[3])});
      }
      grp[q].swap(keep);
    }
  }
  c->tl_cnt[5] = (int)(grp4.size() / 4);
  grp4.insert(grp4.end(), grp4x.begin(), grp4x.end());
  size_t nt = grp4.size() / 4;
  for (int q = 0; q < 4; ++q) nt += grp[q].size() / 4;
  if (nt > c->max_tiles) return fail(c, FDTD_EINVAL, "tile list larger than its reservation");
  hipError_t e = hipStreamSynchronize(c->stream);  // a previous upload may still read c->tl
  if (e != hipSuccess) return hip_fail(c, e, "tile list");
  c->tl.clear();
  c->tl_cnt[4] = (int)(grp4.size() / 4);
  for (int q = 0; q < 4; ++q) {
    c->tl.insert(c->tl.end(), grp[q].begin(), grp[q].end());
    c->tl_cnt[q] = (int)(grp[q].size() / 4);
  }
  c->tl.insert(c->tl.end(), grp4.begin(), grp4.end());
  e = hipMemcpyAsync(c->ws + c->off_tiles, c->tl.data(), c->tl.size() * sizeof(int), hipMemcpyHostToDevice,
                     c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "tile list upload");
  c->tl_var = variant;
  c->tl_ty = ty;
  c->tl_kz = kz;
  return FDTD_OK;
}

// The launches of one step (or one two-step pass) on stream st.  step is the
// absolute step for an eager launch, or the offset from the device counter
// dstep for a launch captured into a graph.  With slot >= 0 the end event of
// the update kernels is recorded before the probes.
int launch_pass(fdtd_ctx* c, hipStream_t st, int variant, bool lists, int lty, int step, const int* dstep, int slot) {
  const int in = c->cur, out = variant == FDTD_KERNEL_SPLIT ? c->cur : 1 - c->cur;
  GridView<float> v32 = c->v32[in][out], p32 = c->v32[out][out];
  GridView<double> v64 = c->v64[in][out], p64 = c->v64[out][out];
  v32.dstep = p32.dstep = dstep;
  v64.dstep = p64.dstep = dstep;
  const bool d64 = c->P.precision == 64;
  const void* view = d64 ? (const void*)&v64 : (const void*)&v32;
  const void* pview = d64 ? (const void*)&p64 : (const void*)&p32;
  int e;
  // Oblique wires: the currents of the pass's (first) step from its input E
  // and their source amplitudes; for a two-step pass also E^{n+1} at the
  // touched edges, the currents of the second step from it, and their
  // amplitudes.  Over tile lists they run on the second stream, ahead of
  // the tiles that read the amplitudes (group 4), beside the others.
  auto wires = [&](hipStream_t ws) -> int {
    const int p = c->P.precision, c16 = c->cls16;
    const OWireView* w = &c->ow_view;
    int r = launch_owire_iq(p, view, w, step, 0, (void*)ws);
    if (!r) r = launch_owire_amp(p, view, c16, w, step, (void*)ws);
    if (!r && variant == FDTD_KERNEL_TB2) {
      r = launch_owire_e1(p, view, c16, w, step, (void*)ws);
      if (!r) r = launch_owire_iq(p, view, w, step + 1, 1, (void*)ws);
      if (!r) r = launch_owire_amp(p, view, c16, w, step + 1, (void*)ws);
    }
    if (r) return fail(c, FDTD_EDEVICE, std::string("oblique-wire launch: ") + hipGetErrorString((hipError_t)r));
    return FDTD_OK;
  };
  if (!c->owr.empty() && !lists) {
    int rc = wires(st);
    if (rc) return rc;
  }
  DebyeView<float> d32 = c->d32;
  DebyeView<double> d64v = c->d64;
  const void* dview = d64 ? (const void*)&d64v : (const void*)&d32;
  if (lists) {
    hipError_t he = hipEventRecord(c->ev_fork, st);
    if (he == hipSuccess) he = hipStreamWaitEvent(c->aux, c->ev_fork, 0);
    if (he != hipSuccess) return hip_fail(c, he, "stream fork");
    if (!c->owr.empty()) {
      he = hipStreamWaitEvent(c->aux2, c->ev_fork, 0);
      if (he != hipSuccess) return hip_fail(c, he, "stream fork");
      int rc = wires(c->aux2);
      if (rc) return rc;
      he = hipEventRecord(c->ev_src, c->aux2);
      if (he != hipSuccess) return hip_fail(c, he, "wire event");
    }
    void* ev_src = c->owr.empty() ? nullptr : (void*)c->ev_src;
    if (c->npole)
      e = launch_fused_debye(c->P.precision, view, dview, c->cls16, step, c->tile_z, c->ws + c->off_tiles,
                             c->tl_cnt, (void*)st, (void*)c->aux);
    else
      e = launch_lists_step(c->P.precision, view, c->cls16, variant, step, lty, c->ws + c->off_tiles, c->tl_cnt,
                            (void*)st, (void*)c->aux, ev_src);
    if (!e) {
      he = hipEventRecord(c->ev_join, c->aux);
      if (he == hipSuccess) he = hipStreamWaitEvent(st, c->ev_join, 0);
      if (he != hipSuccess) return hip_fail(c, he, "stream join");
    }
  } else if (c->npole) {
    e = variant == FDTD_KERNEL_SPLIT
            ? launch_step_debye(c->P.precision, view, dview, c->cls16, step, (void*)st)
            : launch_fused_debye(c->P.precision, view, dview, c->cls16, step, c->tile_z, nullptr, nullptr, (void*)st,
                                 nullptr);
  } else {
    e = launch_step(c->P.precision, view, c->cls16, variant, step, c->tile_y, c->tile_z, (void*)st);
  }
  if (e) return fail(c, FDTD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString((hipError_t)e));
  if (slot >= 0) {  // the timed span ends with the update kernels
    hipError_t he = hipEventRecord(c->ev1[slot], st);
    if (he != hipSuccess) return hip_fail(c, he, "hipEventRecord");
  }
  if (variant == FDTD_KERNEL_TB2)
    e = launch_probes2(c->P.precision, view, c->cls16, step, lists ? 0 : 1, (void*)st);
  else
    e = launch_probes(c->P.precision, pview, step, (void*)st);
  if (e) return fail(c, FDTD_EDEVICE, std::string("probe launch: ") + hipGetErrorString((hipError_t)e));
  return FDTD_OK;
}

void drop_graphs(fdtd_ctx* c) {
  for (int q = 0; q < 2; ++q) {
    if (c->gexec[q]) (void)hipGraphExecDestroy(c->gexec[q]);
    if (c->graph[q]) (void)hipGraphDestroy(c->graph[q]);
    c->gexec[q] = nullptr;
    c->graph[q] = nullptr;
  }
}

// Capture graph_steps steps from the current field-set parity: step offsets
// 0 .. G-1 from the device counter, the ping-pong sets in the order the
// eager loop would use them (G is a multiple of 4, so the parity returns).
int capture_graph(fdtd_ctx* c, int variant, bool lists, int lty) {
  if (!c->cap_stream) {  // the legacy default stream cannot be captured
    hipError_t he = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail(c, he, "capture stream");
  }
  const int cur0 = c->cur, G = c->graph_steps, adv = variant == FDTD_KERNEL_TB2 ? 2 : 1;
  const int* dstep = (const int*)(c->ws + c->off_dstep);
  hipError_t he = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return hip_fail(c, he, "begin capture");
  int rc = FDTD_OK;
  for (int off = 0; off < G && rc == FDTD_OK; off += adv) {
    rc = launch_pass(c, c->cap_stream, variant, lists, lty, off, dstep, -1);
    if (variant != FDTD_KERNEL_SPLIT) c->cur ^= 1;
  }
  c->cur = cur0;
  hipGraph_t gr = nullptr;
  he = hipStreamEndCapture(c->cap_stream, &gr);
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (he != hipSuccess) return hip_fail(c, he, "end capture");
  c->graph[cur0] = gr;
  he = hipGraphInstantiate(&c->gexec[cur0], gr, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    drop_graphs(c);
    return hip_fail(c, he, "graph instantiate");
  }
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_step(fdtd_ctx* c, int n) {
  if (!c || n < 0) return fail(c, FDTD_EINVAL, "bad step count");
  if (!c->ws) return fail(c, FDTD_ESTATE, "no workspace bound");
  if (c->steps_done + n > c->P.max_steps) return fail(c, FDTD_ERANGE, "beyond max_steps");
  // AUTO: the two-step pass over CPML tile lists for grids with a CPML (the
  // fastest on such grids), the fused pass otherwise.  The two-step tiles hold
  // the z CPML table in LDS: thicker layers take the fused pass.
  const bool listable = c->P.npml > 0 && c->N[0] < 65536 && c->N[1] < 65536;
  const bool tb2_ok = tb2_cpml_fits(c->P.npml, c->P.precision);
  int chosen = c->variant != FDTD_KERNEL_AUTO ? c->variant : listable ? FDTD_KERNEL_TB2 : FDTD_KERNEL_FUSED;
  if (chosen == FDTD_KERNEL_TB2 && !tb2_ok) chosen = FDTD_KERNEL_FUSED;
  if (c->npole && !c->owr.empty()) return fail(c, FDTD_EINVAL, "oblique wires in a grid with Debye media");
  // Debye media: the split pass, or the fused pass when asked for (the pole
  // currents would have to live across the two-step pass's stages).  The
  // fused pass with pole currents ran 1% faster than the split pass on
  // 512 x 512 x 384 cells and slower on every smaller grid measured (its
  // CPML slab groups dominate there).
  if (c->npole) chosen = c->variant == FDTD_KERNEL_FUSED ? FDTD_KERNEL_FUSED : FDTD_KERNEL_SPLIT;
  const int lty = c->npole ? 8 : c->tile_y == 4 ? 4 : (c->tile_y == 12 && chosen == FDTD_KERNEL_TB2) ? 12 : 8;
  const int G = c->graph_steps;
  const long long key = ((long long)chosen * 16 + lty) * 65536 + c->tile_z;
  if (G > 0 && key != c->graph_key) {
    drop_graphs(c);
    c->graph_key = key;
  }
  for (int t = 0; t < n;) {
    // the two-step pass needs two steps; an odd remainder takes one fused step
    const int variant = (chosen == FDTD_KERNEL_TB2 && n - t < 2) ? FDTD_KERNEL_FUSED : chosen;
    const int adv = variant == FDTD_KERNEL_TB2 ? 2 : 1;
    // grids with a CPML run the fused and two-step passes over tile lists
    const bool lists = (variant == FDTD_KERNEL_FUSED || variant == FDTD_KERNEL_TB2) && listable;
    const int lkz = std::max(8, c->tile_z > 0 ? c->tile_z : (variant == FDTD_KERNEL_TB2 ? 20 : 32));
    // 12-row tiles exist for the two-step pass only (an odd last step's fused
    // pass takes 8 rows)
    // (Debye grids: 8 rows)
    const int vty = c->npole ? 8 : c->tile_y == 4 ? 4 : (c->tile_y == 12 && variant == FDTD_KERNEL_TB2) ? 12 : 8;
    if (lists) {
      int rc = ensure_tiles(c, variant, vty, lkz);
      if (rc) return rc;
      if (!c->aux) {
        hipError_t he = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (he == hipSuccess && !c->owr.empty()) he = hipStreamCreateWithFlags(&c->aux2, hipStreamNonBlocking);
        if (he == hipSuccess && !c->owr.empty()) he = hipEventCreateWithFlags(&c->ev_src, hipEventDisableTiming);
        if (he != hipSuccess) return hip_fail(c, he, "second stream");
      }
    }
    const bool replay = G > 0 && n - t >= G && variant == chosen;
    int slot = -1;
    if (c->timing) {
      slot = c->ev_next;
      if (c->ev_pending == fdtd_ctx::kRing) {  // drain the oldest pair before reuse
        float ms = 0;
        hipError_t e = hipEventSynchronize(c->ev1[slot]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0[slot], c->ev1[slot]);
        if (e != hipSuccess) return hip_fail(c, e, "kernel timing");
        c->timed_ms += ms;
        c->timed_steps += c->ev_steps[slot];
        --c->ev_pending;
      }
    }
    int e;
    if (replay) {
      if (!c->gexec[c->cur]) {
        int rc = capture_graph(c, variant, lists, vty);
        if (rc) return rc;
      }
      e = launch_set((int*)(c->ws + c->off_dstep), (int)c->steps_done, (void*)c->stream);
      if (e) return fail(c, FDTD_EDEVICE, std::string("step counter: ") + hipGetErrorString((hipError_t)e));
      if (slot >= 0 && hipEventRecord(c->ev0[slot], c->stream) != hipSuccess) return fail(c, FDTD_EDEVICE, "event");
      hipError_t he = hipGraphLaunch(c->gexec[c->cur], c->stream);
      if (he != hipSuccess) return hip_fail(c, he, "graph launch");
    } else {
      if (slot >= 0 && hipEventRecord(c->ev0[slot], c->stream) != hipSuccess) return fail(c, FDTD_EDEVICE, "event");
      int rc = launch_pass(c, c->stream, variant, lists, vty, (int)c->steps_done, nullptr, slot);
      if (rc) return rc;
    }
    const int done = replay ? G : adv;
    if (!replay && variant != FDTD_KERNEL_SPLIT) c->cur ^= 1;
    if (slot >= 0) {
      if (replay) {  // a replayed graph is timed whole, its probe launches included
        hipError_t er = hipEventRecord(c->ev1[slot], c->stream);
        if (er != hipSuccess) return hip_fail(c, er, "hipEventRecord");
      }
      c->ev_steps[slot] = done;
      c->ev_next = (slot + 1) % fdtd_ctx::kRing;
      ++c->ev_pending;
    }
    c->steps_done += done;
    t += done;
  }
  return FDTD_OK;
}

int fdtd_set_graph(fdtd_ctx* c, int graph_steps) {
  if (!c) return FDTD_EINVAL;
  if (graph_steps < 0 || graph_steps % 4) return fail(c, FDTD_EINVAL, "graph_steps must be a multiple of 4 (0: off)");
  if (graph_steps != c->graph_steps) drop_graphs(c);
  c->graph_steps = graph_steps;
  return FDTD_OK;
}

int fdtd_timing(fdtd_ctx* c, int enable) {
  if (!c) return FDTD_EINVAL;
  if (enable && !c->ev0[0]) {
    for (int q = 0; q < fdtd_ctx::kRing; ++q) {
      hipError_t e = hipEventCreate(&c->ev0[q]);
      if (e == hipSuccess) e = hipEventCreate(&c->ev1[q]);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
  }
  c->timing = enable != 0;
  return FDTD_OK;
}

int fdtd_kernel_time(fdtd_ctx* c, double* total_ms, long long* n_steps) {
  if (!c || !total_ms || !n_steps) return FDTD_EINVAL;
  while (c->ev_pending > 0) {
    const int slot = (c->ev_next - c->ev_pending + fdtd_ctx::kRing) % fdtd_ctx::kRing;
    float ms = 0;
    hipError_t e = hipEventSynchronize(c->ev1[slot]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0[slot], c->ev1[slot]);
    if (e != hipSuccess) return hip_fail(c, e, "kernel timing");
    c->timed_ms += ms;
    c->timed_steps += c->ev_steps[slot];
    --c->ev_pending;
  }
  *total_ms = c->timed_ms;
  *n_steps = c->timed_steps;
  c->timed_ms = 0;
  c->timed_steps = 0;
  return FDTD_OK;
}

int fdtd_probe(fdtd_ctx* c, int id, double* out, int n_max, int* n_written) {
  if (!c || !out || id < 0 || id >= (int)c->probes.size() || n_max < 0) return fail(c, FDTD_EINVAL, "bad probe");
  if (!c->ws) return fail(c, FDTD_ESTATE, "no workspace bound");
  const int n = (int)std::min<long long>(c->steps_done, n_max);
  const double* src = (const double*)(c->ws + c->off_out) + (size_t)id * c->P.max_steps;
  hipError_t e = hipMemcpyAsync(out, src, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "probe copy");
  if (n_written) *n_written = n;
  if (!finite_all(out, (size_t)n)) return fail(c, FDTD_ENONFINITE, "probe record holds NaN or Inf");
  return FDTD_OK;
}

static int field_ptr(fdtd_ctx* c, int comp, char** p) {
  if (comp < 0 || comp > 5) return FDTD_EINVAL;
  const size_t ts = tsize(c);
  *p = c->ws + c->off_f + ((size_t)(c->cur * 6 + comp)) * (size_t)c->ncell * ts;
  return FDTD_OK;
}

int fdtd_set_field(fdtd_ctx* c, int comp, const double* host) {
  if (!c || !host || comp < 0 || comp > 5) return fail(c, FDTD_EINVAL, "bad field arguments");
  if (!c->ws) return fail(c, FDTD_ESTATE, "no workspace bound");
  char* dst;
  field_ptr(c, comp, &dst);
  const size_t N = (size_t)c->ncell;
  std::vector<double> v(host, host + N);
  if (comp < 3)  // perfect-conductor edges (walls, wires) have Cb = 0
    for (size_t n = 0; n < N; ++n)
      if (c->ctab[(size_t)c->cls_id[n] * K_NCOEF + 2 * comp + 1] == 0.0) v[n] = 0.0;
  hipError_t e;
  if (c->P.precision == 64) {
    e = hipMemcpyAsync(dst, v.data(), N * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    std::vector<float> f(v.begin(), v.end());
    e = hipMemcpyAsync(dst, f.data(), N * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "set_field");
  return FDTD_OK;
}

int fdtd_get_field(fdtd_ctx* c, int comp, double* host) {
  if (!c || !host || comp < 0 || comp > 5) return fail(c, FDTD_EINVAL, "bad field arguments");
  if (!c->ws) return fail(c, FDTD_ESTATE, "no workspace bound");
  char* src;
  field_ptr(c, comp, &src);
  const size_t N = (size_t)c->ncell;
  hipError_t e;
  if (c->P.precision == 64) {
    e = hipMemcpyAsync(host, src, N * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    std::vector<float> f(N);
    e = hipMemcpyAsync(f.data(), src, N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    for (size_t n = 0; n < N; ++n) host[n] = f[n];
  }
  if (e != hipSuccess) return hip_fail(c, e, "get_field");
  return FDTD_OK;
}

double fdtd_dt(const fdtd_ctx* c) { return c ? c->dt : 0.0; }
long long fdtd_steps_done(const fdtd_ctx* c) { return c ? c->steps_done : -1; }
int fdtd_num_classes(const fdtd_ctx* c) { return c ? c->ncls : -1; }

double fdtd_algorithmic_bytes_per_step(const fdtd_ctx* c) {
  if (!c) return 0.0;
  const double ts = c->P.precision == 64 ? 8.0 : 4.0;
  double b = (double)c->ncell * (12.0 * ts + (c->cls16 ? 2.0 : 1.0));
  // each CPML slab cell reads and writes 4 psi values per axis it lies in
  for (int u = 0; u < 3; ++u) b += (double)c->psi_elems[u] * 4.0 * 2.0 * ts;
  // (psi_elems counts the whole 2 npml slab pair of an axis)
  // a node with Debye poles reads and writes one current per component and pole
  b += (double)c->debye_nodes * 3.0 * c->npole * 2.0 * ts;
  return b;
}

const char* fdtd_last_error(const fdtd_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ===========================================================================
// Batched engine: many independent grids stepped together.
// ===========================================================================

struct fdtd_batch {
  std::vector<fdtd_ctx*> grids;
  hipStream_t stream = nullptr;
  int prec = 32, cls16 = 0, pml = 0;
  int tx = 32, ty = 8, kz = 32;
  int max_steps = 0;
  std::string err;
  // layout
  std::vector<size_t> off;            // sub-workspace of each grid
  size_t off_views = 0, off_pviews = 0, off_tiles = 0, off_plist = 0, off_step = 0, ws_bytes = 0;
  std::vector<int> tiles;             // int4 entries (grid, i0, j0, k0 | kz << 16)
  std::vector<int> plist;             // int2 entries (grid, probe)
  // two-step passes (set_kernel with tile_x 60): CPML-grouped tile list of
  // (grid, i0 | iw << 16, j0 | jh << 16, k0 | kz << 16); an odd remainder of
  // steps takes one fused step over `tiles` (32 x 8)
  bool tb2 = false;
  int tb2_kz = 32;
  std::vector<int> tiles2;
  int tcnt[4] = {0, 0, 0, 0};
  size_t off_tiles2 = 0;
  // the same tiles for the persistent launches (fdtd_batch_set_persistent):
  // one list per code path (x-slab instantiation, then all-axes), each grid
  // by grid, tagged with their group, in 8 runs (one per XCD), and the runs'
  // 2 x 8 counters
  bool persistent = true;
  std::vector<int> tiles_q;
  QRuns runs[2] = {};
  int nq[2] = {0, 0};
  int q_blocks[2] = {0, 0};
  size_t off_tiles_q = 0, off_qctr = 0;
  char* ws = nullptr;
  int cur = 0;
  long long steps_done = 0;
  bool tiles_dirty = true;
  // graph replay (captured on a private stream, launched on `stream`)
  hipStream_t cap_stream = nullptr;
  // second stream of the two-step pass (the x-slab tile group beside the rest)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int graph_steps = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_tiles = -1;
  // timing
  bool timing = false;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  double timed_ms = 0;
  long long timed_steps = 0;
};

namespace {

int bfail(fdtd_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

size_t view_bytes(int prec) { return prec == 64 ? sizeof(GridView<double>) : sizeof(GridView<float>); }

// Tile list: every grid cut into tx x ty x kz tiles; larger grids first so
// the long-running tiles start early (longest-processing-time order).
void build_tiles(fdtd_batch* b) {
  std::vector<int> order(b->grids.size());
  for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->grids[a]->ncell > b->grids[c]->ncell; });
  b->tiles.clear();
  for (int g : order) {
    const fdtd_ctx* c = b->grids[g];
    for (int k0 = 0; k0 < c->N[2]; k0 += b->kz)
      for (int j0 = 0; j0 < c->N[1]; j0 += b->ty)
        for (int i0 = 0; i0 < c->N[0]; i0 += b->tx) {
          b->tiles.push_back(g);
          b->tiles.push_back(i0);
          b->tiles.push_back(j0);
          b->tiles.push_back(k0 | (b->kz << 16));
        }
  }
}

// Two-step tile list of every grid, grouped by the CPML slabs the tiles reach
// (as for a single grid), larger grids first within each group.
void build_tiles_tb2(fdtd_batch* b) {
  std::vector<int> order(b->grids.size());
  for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->grids[a]->ncell > b->grids[c]->ncell; });
  std::vector<int> grp[4];
  const int kz = b->tb2_kz, kzp = std::max(8, kz / 2);
  for (int g : order) {
    const fdtd_ctx* c = b->grids[g];
    const int np = c->P.npml, nz = c->N[2];
    const std::vector<Seg> xs = segments_tb2(c->N[0], np, 60, 2);
    const std::vector<Seg> ys = segments_tb2(c->N[1], np, 8, 2);
    for (const Seg& y : ys)
      for (const Seg& x : xs) {
        const int q = (x.in ? 0 : 1) | (y.in ? 0 : 2);
        const int d = q == 0 ? kz : kzp;
        for (int z = 0; z < nz; z += d)
          grp[q].insert(grp[q].end(), {g, x.a | (x.b - x.a) << 16, y.a | (y.b - y.a) << 16,
                                       z | (std::min(d, nz - z) << 16)});
      }
  }
  b->tiles2.clear();
  for (int q = 0; q < 4; ++q) {
    b->tiles2.insert(b->tiles2.end(), grp[q].begin(), grp[q].end());
    b->tcnt[q] = (int)(grp[q].size() / 4);
  }
  // Persistent lists: the same tiles grid by grid (in the order above), the
  // group in the top byte of the grid field; list 0 for the x-slab code path
  // (groups 0 and 1), list 1 for the all-axes one (groups 2 and 3; every
  // tile in FP64); each cut into 8 runs of about equal cell count.
  std::vector<std::vector<int>> per(b->grids.size());
  for (int q = 0; q < 4; ++q)
    for (size_t t = 0; t < grp[q].size(); t += 4)
      per[grp[q][t]].insert(per[grp[q][t]].end(), {grp[q][t] | (q << 24), grp[q][t + 1], grp[q][t + 2],
                                                   grp[q][t + 3]});
  std::vector<int> lst[2];
  std::vector<double> cells[2];
  double total[2] = {0, 0};
  for (int g : order)
    for (size_t t = 0; t < per[g].size(); t += 4) {
      const int* e = &per[g][t];
      const int w = (b->prec == 64 || ((e[0] >> 24) & 2)) ? 1 : 0;
      lst[w].insert(lst[w].end(), e, e + 4);
      cells[w].push_back((double)(e[1] >> 16) * (e[2] >> 16) * (e[3] >> 16));
      total[w] += cells[w].back();
    }
  b->tiles_q = lst[0];
  b->tiles_q.insert(b->tiles_q.end(), lst[1].begin(), lst[1].end());
  for (int w = 0; w < 2; ++w) {
    const int n = (int)cells[w].size();
    QRuns& r = b->runs[w];
    b->nq[w] = n;
    r.start[0] = 0;
    double acc = 0;
    int x = 1;
    for (int t = 0; t < n && x < 8; ++t) {
      acc += cells[w][t];
      while (x < 8 && acc >= total[w] * x / 8.0) r.start[x++] = t + 1;
    }
    while (x <= 8) r.start[x++] = n;
  }
}

template <typename T>
int batch_upload(fdtd_batch* b) {
  const size_t nv = b->grids.size();
  std::vector<GridView<T>> views(2 * nv), pviews(2 * nv);
  for (size_t g = 0; g < nv; ++g) {
    fdtd_ctx* c = b->grids[g];
    for (int p = 0; p < 2; ++p) {
      views[p * nv + g] = view_of<T>(c, p, 1 - p);       // step reading set p
      pviews[p * nv + g] = view_of<T>(c, 1 - p, 1 - p);  // probes after it
    }
  }
  hipError_t e = hipMemcpyAsync(b->ws + b->off_views, views.data(), views.size() * sizeof(GridView<T>),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->off_pviews, pviews.data(), pviews.size() * sizeof(GridView<T>),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && !b->plist.empty())
    e = hipMemcpyAsync(b->ws + b->off_plist, b->plist.data(), b->plist.size() * sizeof(int),
                       hipMemcpyHostToDevice, b->stream);
  const int zero = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(b->ws + b->off_step, &zero, sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("batch upload: ") + hipGetErrorString(e));
  return FDTD_OK;
}

int upload_tiles(fdtd_batch* b) {
  build_tiles(b);
  hipError_t e = hipMemcpyAsync(b->ws + b->off_tiles, b->tiles.data(), b->tiles.size() * sizeof(int),
                                hipMemcpyHostToDevice, b->stream);
  if (b->tb2 && e == hipSuccess) {
    build_tiles_tb2(b);
    e = hipMemcpyAsync(b->ws + b->off_tiles2, b->tiles2.data(), b->tiles2.size() * sizeof(int),
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->ws + b->off_tiles_q, b->tiles_q.data(), b->tiles_q.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !b->q_blocks[0]) {
      b->q_blocks[0] = batch_queue_blocks(b->prec, b->cls16, 5);
      b->q_blocks[1] = batch_queue_blocks(b->prec, b->cls16, 7);
      if (b->q_blocks[0] <= 0 || b->q_blocks[1] <= 0) return bfail(b, FDTD_EDEVICE, "persistent launch size");
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("tile upload: ") + hipGetErrorString(e));
  b->tiles_dirty = false;
  return FDTD_OK;
}

size_t max_tiles(const fdtd_batch* b) {  // upper bound over the allowed tile shapes
  size_t n = 0;
  for (const fdtd_ctx* c : b->grids)
    n += (size_t)((c->N[0] + 31) / 32) * ((c->N[1] + 7) / 8) * ((c->N[2] + 7) / 8);
  return n;
}

size_t max_tiles_tb2(const fdtd_batch* b) {  // 60 x 8 pieces (3 extra per axis), chunks of >= 8 planes
  size_t n = 0;
  for (const fdtd_ctx* c : b->grids) n += (size_t)(c->N[0] / 60 + 3) * (c->N[1] / 8 + 3) * (c->N[2] / 8 + 1);
  return n;
}

// One two-step pass (kernels + probes of both steps) on stream `st`, steps
// *d_step + off and + 1; parity p selects the view tables.
int batch_launch_pass(fdtd_batch* b, hipStream_t st, int p, int off) {
  const size_t nv = b->grids.size();
  const size_t vb = view_bytes(b->prec);
  const int* d_step = (const int*)(b->ws + b->off_step);
  if (b->persistent) {
    const int* tq = (const int*)(b->ws + b->off_tiles_q);
    int e = launch_batch_pass_queue(b->prec, b->cls16, b->ws + b->off_views + p * nv * vb, tq, &b->runs[0],
                                    std::min(b->q_blocks[0], b->nq[0]), tq + 4 * b->nq[0], &b->runs[1],
                                    std::min(b->q_blocks[1], b->nq[1]), (int*)(b->ws + b->off_qctr),
                                    b->ws + b->off_plist, (int)(b->plist.size() / 2), d_step, off, (void*)st,
                                    (void*)b->aux, (void*)b->ev_fork, (void*)b->ev_join);
    if (e) return bfail(b, FDTD_EDEVICE, std::string("batch pass: ") + hipGetErrorString((hipError_t)e));
    return FDTD_OK;
  }
  int e = launch_batch_pass_tb2(b->prec, b->cls16, b->ws + b->off_views + p * nv * vb, b->ws + b->off_tiles2,
                                b->tcnt, b->ws + b->off_plist, (int)(b->plist.size() / 2), d_step, off, (void*)st,
                                (void*)b->aux, (void*)b->ev_fork, (void*)b->ev_join);
  if (e) return bfail(b, FDTD_EDEVICE, std::string("batch pass: ") + hipGetErrorString((hipError_t)e));
  return FDTD_OK;
}

// Launch one step (kernel + probes) on stream `st` with step offset `off`
// relative to the device counter; parity p selects the view tables.
int batch_launch_step(fdtd_batch* b, hipStream_t st, int p, int off) {
  const size_t nv = b->grids.size();
  const size_t vb = view_bytes(b->prec);
  const int* d_step = (const int*)(b->ws + b->off_step);
  int e = launch_batch_step(b->prec, b->cls16, b->pml, b->ws + b->off_views + p * nv * vb, b->ws + b->off_tiles,
                            (int)(b->tiles.size() / 4), b->tx, b->ty, d_step, off, (void*)st);
  if (e) return bfail(b, FDTD_EDEVICE, std::string("batch kernel: ") + hipGetErrorString((hipError_t)e));
  e = launch_batch_probes(b->prec, b->ws + b->off_pviews + p * nv * vb, b->ws + b->off_plist,
                          (int)(b->plist.size() / 2), d_step, off, (void*)st);
  if (e) return bfail(b, FDTD_EDEVICE, std::string("batch probes: ") + hipGetErrorString((hipError_t)e));
  return FDTD_OK;
}

void drop_graph(fdtd_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

int fdtd_batch_pack(fdtd_ctx* const* grids, int n, void* hip_stream, fdtd_batch** out) {
  if (!grids || n < 1 || !out) return FDTD_EINVAL;
  *out = nullptr;
  fdtd_batch* b = new fdtd_batch;
  b->stream = (hipStream_t)hip_stream;
  b->max_steps = 1 << 30;
  for (int g = 0; g < n; ++g) {
    fdtd_ctx* c = grids[g];
    if (!c) { delete b; return FDTD_EINVAL; }
    int rc = freeze(c);
    if (rc) { delete b; return rc; }
    if (c->ws) { delete b; return FDTD_ESTATE; }  // already bound on its own
    if (c->npole || !c->owr.empty()) { delete b; return FDTD_EINVAL; }  // Debye media, oblique wires: split pass on their own
    if (g == 0) {
      b->prec = c->P.precision;
      b->cls16 = c->cls16;
      b->pml = c->P.npml > 0;
    } else if (c->P.precision != b->prec || c->cls16 != b->cls16 || (c->P.npml > 0) != (b->pml != 0)) {
      delete b;
      return FDTD_EINVAL;  // one kernel instantiation serves the whole batch
    }
    b->max_steps = std::min(b->max_steps, c->P.max_steps);
    b->grids.push_back(c);
    for (size_t q = 0; q < c->probes.size(); ++q) {
      b->plist.push_back(g);
      b->plist.push_back((int)q);
    }
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  for (fdtd_ctx* c : b->grids) b->off.push_back(take(c->ws_bytes));
  b->off_views = take(2 * b->grids.size() * view_bytes(b->prec));
  b->off_pviews = take(2 * b->grids.size() * view_bytes(b->prec));
  b->off_tiles = take(max_tiles(b) * 4 * sizeof(int));
  b->off_tiles2 = take(max_tiles_tb2(b) * 4 * sizeof(int));
  b->off_tiles_q = take(max_tiles_tb2(b) * 4 * sizeof(int));
  b->off_qctr = take(16 * sizeof(int));
  b->off_plist = take(b->plist.size() * sizeof(int) + 8);
  b->off_step = take(sizeof(int));
  b->ws_bytes = o;
  *out = b;
  return FDTD_OK;
}

size_t fdtd_batch_workspace_bytes(const fdtd_batch* b) { return b ? b->ws_bytes : 0; }

int fdtd_batch_bind_workspace(fdtd_batch* b, void* dev, size_t bytes) {
  if (!b) return FDTD_EINVAL;
  if (b->ws) return bfail(b, FDTD_ESTATE, "batch workspace already bound");
  if (!dev || bytes < b->ws_bytes) return bfail(b, FDTD_ENOMEM, "batch workspace too small");
  if (((uintptr_t)dev & 255) != 0) return bfail(b, FDTD_ENOMEM, "batch workspace not 256-byte aligned");
  b->ws = (char*)dev;
  for (size_t g = 0; g < b->grids.size(); ++g) {
    fdtd_ctx* c = b->grids[g];
    c->stream = b->stream;
    c->ws = b->ws + b->off[g];
    int rc = b->prec == 64 ? upload<double>(c) : upload<float>(c);
    if (rc) { b->ws = nullptr; return bfail(b, rc, "grid " + std::to_string(g) + ": " + c->err); }
  }
  int rc = b->prec == 64 ? batch_upload<double>(b) : batch_upload<float>(b);
  if (rc) return rc;
  return upload_tiles(b);
}

int fdtd_batch_set_kernel(fdtd_batch* b, int tile_x, int tile_y, int tile_z, int graph_steps) {
  if (!b) return FDTD_EINVAL;
  if (tile_x == 60) {  // two-step passes
    if (tile_y != 8 || tile_z < 16 || tile_z > 4096 || graph_steps < 0 || (graph_steps % 4))
      return bfail(b, FDTD_EINVAL, "two-step tiles (60, 8), tile_z in [16, 4096], graph_steps a multiple of 4");
    for (const fdtd_ctx* c : b->grids)
      if (!tb2_cpml_fits(c->P.npml, c->P.precision))
        return bfail(b, FDTD_EINVAL, "two-step tiles need 2 npml <= 128 (FP32) or 64 (FP64)");
    b->tb2 = true;
    b->tb2_kz = tile_z;
    b->tx = 32;
    b->ty = 8;
    b->kz = 32;
    b->graph_steps = graph_steps;
    b->tiles_dirty = true;
    drop_graph(b);
    return FDTD_OK;
  }
  const bool ok = (tile_x == 32 && (tile_y == 8 || tile_y == 16)) || (tile_x == 64 && tile_y == 8);
  if (!ok || tile_z < 8 || tile_z > 4096 || graph_steps < 0 || (graph_steps & 1))
    return bfail(b, FDTD_EINVAL, "tiles (32, 8|16), (64, 8) or (60, 8), tile_z in [8, 4096], even graph_steps");
  b->tb2 = false;
  b->tx = tile_x;
  b->ty = tile_y;
  b->kz = tile_z;
  b->graph_steps = graph_steps;
  b->tiles_dirty = true;
  drop_graph(b);
  return FDTD_OK;
}

int fdtd_batch_set_persistent(fdtd_batch* b, int on) {
  if (!b || (on != 0 && on != 1)) return FDTD_EINVAL;
  if (b->persistent != (on == 1)) drop_graph(b);
  b->persistent = on == 1;
  return FDTD_OK;
}

int fdtd_batch_run(fdtd_batch* b, int n) {
  if (!b || n < 0) return FDTD_EINVAL;
  if (!b->ws) return bfail(b, FDTD_ESTATE, "no batch workspace bound");
  if (b->steps_done + n > b->max_steps) return bfail(b, FDTD_ERANGE, "beyond max_steps");
  if (b->tiles_dirty) {
    int rc = upload_tiles(b);
    if (rc) return rc;
  }
  hipError_t e = hipSuccess;
  if (b->tb2 && !b->aux) {  // the two-step pass's second stream, made outside any capture
    e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("second stream: ") + hipGetErrorString(e));
  }
  if (b->timing) {
    if (!b->t0) {
      e = hipEventCreate(&b->t0);
      if (e == hipSuccess) e = hipEventCreate(&b->t1);
    }
    if (e == hipSuccess) e = hipEventRecord(b->t0, b->stream);
    if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, hipGetErrorString(e));
  }
  int left = n;
  const int G = b->graph_steps;
  while (left > 0) {
    if (G > 0 && left >= G && b->cur == 0) {
      if (!b->gexec) {  // capture G steps once: offsets 0..G-1, then advance the counter by G
        if (!b->cap_stream) {  // the legacy default stream cannot be captured
          e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
          if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("capture stream: ") + hipGetErrorString(e));
        }
        hipStream_t cs = b->cap_stream;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        int rc = FDTD_OK;
        if (b->tb2)
          for (int t = 0; t < G / 2 && rc == FDTD_OK; ++t) rc = batch_launch_pass(b, cs, t & 1, 2 * t);
        else
          for (int t = 0; t < G && rc == FDTD_OK; ++t) rc = batch_launch_step(b, cs, t & 1, t);
        if (rc == FDTD_OK && launch_add((int*)(b->ws + b->off_step), G, (void*)cs))
          rc = bfail(b, FDTD_EDEVICE, "capture: counter");
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        if (rc) { if (gr) (void)hipGraphDestroy(gr); return rc; }
        if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("end capture: ") + hipGetErrorString(e));
        b->graph = gr;
        e = hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_graph(b); return bfail(b, FDTD_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e)); }
      }
      e = hipGraphLaunch(b->gexec, b->stream);
      if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
      left -= G;
      b->steps_done += G;
      continue;
    }
    const int adv = (b->tb2 && left >= 2) ? 2 : 1;
    int rc = adv == 2 ? batch_launch_pass(b, b->stream, b->cur, 0) : batch_launch_step(b, b->stream, b->cur, 0);
    if (rc) return rc;
    if (launch_add((int*)(b->ws + b->off_step), adv, (void*)b->stream)) return bfail(b, FDTD_EDEVICE, "counter");
    b->cur ^= 1;
    b->steps_done += adv;
    left -= adv;
  }
  if (b->timing) {
    float ms = 0;
    e = hipEventRecord(b->t1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b->t1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->t0, b->t1);
    if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, hipGetErrorString(e));
    b->timed_ms += ms;
    b->timed_steps += n;
  }
  for (fdtd_ctx* c : b->grids) {  // keep the member contexts consistent
    c->cur = b->cur;
    c->steps_done = b->steps_done;
  }
  return FDTD_OK;
}

int fdtd_batch_timing(fdtd_batch* b, int enable) {
  if (!b) return FDTD_EINVAL;
  b->timing = enable != 0;
  return FDTD_OK;
}

int fdtd_batch_time(fdtd_batch* b, double* total_ms, long long* n_steps) {
  if (!b || !total_ms || !n_steps) return FDTD_EINVAL;
  *total_ms = b->timed_ms;
  *n_steps = b->timed_steps;
  b->timed_ms = 0;
  b->timed_steps = 0;
  return FDTD_OK;
}

int fdtd_batch_probe(fdtd_batch* b, int g, int probe_id, double* out, int n_max, int* n_written) {
  if (!b || g < 0 || g >= (int)b->grids.size()) return FDTD_EINVAL;
  return fdtd_probe(b->grids[g], probe_id, out, n_max, n_written);
}

long long fdtd_batch_cells(const fdtd_batch* b) {
  if (!b) return -1;
  long long n = 0;
  for (const fdtd_ctx* c : b->grids) n += c->ncell;
  return n;
}

double fdtd_batch_algorithmic_bytes_per_step(const fdtd_batch* b) {
  if (!b) return 0.0;
  double s = 0;
  for (const fdtd_ctx* c : b->grids) s += fdtd_algorithmic_bytes_per_step(c);
  return s;
}

const char* fdtd_batch_last_error(const fdtd_batch* b) { return b ? b->err.c_str() : "null batch"; }

void fdtd_batch_destroy(fdtd_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->aux) (void)hipStreamSynchronize(b->aux);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->aux) (void)hipStreamDestroy(b->aux);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->t0) (void)hipEventDestroy(b->t0);
  if (b->t1) (void)hipEventDestroy(b->t1);
  for (fdtd_ctx* c : b->grids) c->ws = nullptr;  // the workspace belonged to the batch
  delete b;
}

void fdtd_destroy(fdtd_ctx* c) {
  if (!c) return;
  if (c->ws) (void)hipStreamSynchronize(c->stream);  // nothing may still use the workspace
  fdtd_static_release(c);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux) (void)hipStreamSynchronize(c->aux);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->aux2) (void)hipStreamSynchronize(c->aux2);
  if (c->ev_src) (void)hipEventDestroy(c->ev_src);
  if (c->aux2) (void)hipStreamDestroy(c->aux2);
  for (int q = 0; q < fdtd_ctx::kRing; ++q) {
    if (c->ev0[q]) (void)hipEventDestroy(c->ev0[q]);
    if (c->ev1[q]) (void)hipEventDestroy(c->ev1[q]);
  }
  delete c;
}

}  // extern "C"
