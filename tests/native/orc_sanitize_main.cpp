// Drives every call of the FP64 oracle (test infrastructure) under the
// address and undefined-behaviour sanitizers: set-up with every element kind,
// stepping with CPML, Debye media, wires, lumped elements, probes, an
// oblique wire in a second grid, field and coefficient reads, and the error
// paths.  Prints "ok" and exits 0 when every call returned what it should.
#include <cmath>
#include <cstdio>
#include <vector>

#include "orc.h"

static int fails = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("expectation failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static orc_params params(int nx, int ny, int nz, int npml, int steps) {
  orc_params p{};
  p.nx = nx; p.ny = ny; p.nz = nz; p.dx = 0.25; p.dt = 0; p.npml = npml;
  p.pml_m = 3; p.pml_sigma_factor = 1; p.pml_kappa_max = 2; p.pml_alpha_max = 0.02; p.pml_ma = 1;
  p.loss_mode = ORC_LOSS_SEMI; p.wire_r0_factor = std::exp(-1.5707963267948966); p.max_steps = steps;
  return p;
}

int main() {
  orc_set_threads(2);
  const int nx = 17, ny = 13, nz = 11, n = 24;
  orc_sim* s = nullptr;
  EXPECT(orc_create(nullptr, &s) != ORC_OK);
  orc_params bad = params(1, ny, nz, 0, n);
  EXPECT(orc_create(&bad, &s) != ORC_OK);
  orc_params p = params(nx, ny, nz, 3, n);
  EXPECT(orc_create(&p, &s) == ORC_OK);
  std::vector<uint8_t> cm((size_t)nx * ny * nz);
  for (size_t i = 0; i < cm.size(); ++i) cm[i] = (uint8_t)(i % 3);
  const orc_material mats[3] = {{1, 0, 1}, {10, 0.01, 1}, {4, 0.002, 2}};
  EXPECT(orc_set_materials(s, cm.data(), mats, 2) != ORC_OK);  // id 2 out of range
  EXPECT(orc_set_materials(s, cm.data(), mats, 3) == ORC_OK);
  const double tau[2] = {1e-9, 2e-8}, deps[6] = {0, 0, 3, 1, 2, 0.5};
  EXPECT(orc_set_debye(s, 2, tau, deps) == ORC_OK);
  EXPECT(orc_add_wire(s, 0, 2, 6, 5, 12, 0.004) == ORC_OK);
  EXPECT(orc_add_wire(s, 3, 2, 6, 5, 12, 0.004) != ORC_OK);     // bad axis
  EXPECT(orc_add_wire(s, 2, 8, 3, 1, 40, 0.004) != ORC_OK);     // beyond the grid
  std::vector<double> amps(n);
  for (int t = 0; t < n; ++t) amps[t] = std::exp(-((t - 8.0) / 3.0) * ((t - 8.0) / 3.0));
  EXPECT(orc_add_source(s, 2, 8, 7, 5, amps.data(), n) == ORC_OK);
  EXPECT(orc_add_source(s, 2, 0, 7, 5, amps.data(), n) != ORC_OK);  // PEC wall edge
  EXPECT(orc_add_lumped(s, ORC_LUMPED_R, 1, 9, 3, 4, 50.0) == ORC_OK);
  EXPECT(orc_add_lumped(s, ORC_LUMPED_C, 1, 9, 3, 4, 1e-10) == ORC_OK);
  EXPECT(orc_add_source_r(s, ORC_SRC_VOLTAGE, 0, 10, 9, 7, amps.data(), n, 25.0) == ORC_OK);
  int pe = -1, pv = -1, pi = -1;
  EXPECT(orc_add_probe(s, ORC_PR_E, 2, 8, 7, 6, 1, &pe) == ORC_OK);
  EXPECT(orc_add_probe(s, ORC_PR_VLINE, 0, 1, 7, 5, 10, &pv) == ORC_OK);
  EXPECT(orc_add_probe(s, ORC_PR_ILOOP, 2, 8, 7, 5, 1, &pi) == ORC_OK);
  EXPECT(orc_add_probe(s, ORC_PR_VLINE, 0, 1, 7, 5, 40, &pv) != ORC_OK);
  EXPECT(orc_step(s, n / 2) == ORC_OK);
  EXPECT(orc_add_wire(s, 1, 3, 2, 2, 3, 0.004) == ORC_ESTATE);   // set-up after stepping
  EXPECT(orc_step(s, n / 2) == ORC_OK);
  EXPECT(orc_step(s, 1) != ORC_OK);                              // beyond max_steps
  std::vector<double> rec(n), field(cm.size());
  int nw = 0;
  EXPECT(orc_probe(s, pe, rec.data(), n, &nw) == ORC_OK && nw == n);
  EXPECT(orc_probe(s, pv, rec.data(), n, &nw) == ORC_OK);
  EXPECT(orc_probe(s, pi, rec.data(), n, &nw) == ORC_OK);
  EXPECT(orc_probe(s, 99, rec.data(), n, &nw) != ORC_OK);
  for (int c = 0; c < 6; ++c) {
    EXPECT(orc_get_field(s, c, field.data()) == ORC_OK);
    for (double v : field) EXPECT(std::isfinite(v));
    EXPECT(orc_set_field(s, c, field.data()) == ORC_OK);
  }
  for (int c = 0; c < 6; ++c) EXPECT(orc_get_coef(s, c, 0, field.data()) == ORC_OK);
  EXPECT(orc_dt(s) > 0 && orc_last_error(s) != nullptr);
  orc_destroy(s);

  // an oblique wire (no Debye media), driven and recorded, in a second grid
  orc_params q = params(20, 20, 20, 2, 40);
  EXPECT(orc_create(&q, &s) == ORC_OK);
  const double a[3] = {3.5, 4.2, 3.1}, b[3] = {15.9, 14.3, 15.8}, far[3] = {30, 4, 4};
  int wid = -1;
  EXPECT(orc_add_oblique_wire(s, a, far, 0.002, -1, nullptr, 0, -1, &wid) != ORC_OK);
  EXPECT(orc_add_oblique_wire(s, a, b, 0.002, 3, amps.data(), n, 5, &wid) == ORC_OK);
  EXPECT(orc_add_oblique_wire(s, a, b, 0.002, 99, amps.data(), n, 5, &wid) != ORC_OK);
  // a second wire from the first one's end, joined there
  const double e[3] = {4.4, 15.6, 9.2};
  int w2 = -1;
  EXPECT(orc_add_oblique_wire(s, b, e, 0.004, -1, nullptr, 0, -1, &w2) == ORC_OK);
  const int ids[2] = {wid, w2}, ends[2] = {1, 0}, mism[2] = {0, 0};
  EXPECT(orc_join_oblique_wires(s, 2, ids, mism) != ORC_OK);        // the two starts do not meet
  EXPECT(orc_join_oblique_wires(s, 2, ids, ends) == ORC_OK);
  EXPECT(orc_join_oblique_wires(s, 2, ids, ends) != ORC_OK);        // already joined
  EXPECT(orc_step(s, 40) == ORC_OK);
  int ns = 0, nr = 0;
  EXPECT(orc_oblique_wire_read(s, wid, nullptr, nullptr, nullptr, 0, &ns, &nr) == ORC_OK && ns > 0);
  std::vector<double> cur(ns), qq(ns + 1), rw(40);
  EXPECT(orc_oblique_wire_read(s, wid, cur.data(), qq.data(), rw.data(), 40, &ns, &nr) == ORC_OK && nr == 40);
  for (double v : cur) EXPECT(std::isfinite(v));
  orc_destroy(s);
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
