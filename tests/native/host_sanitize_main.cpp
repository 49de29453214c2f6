// Drives the host-side set-up of the HIP FDTD library (everything that runs
// before a workspace is bound, so no GPU is needed) under the address and
// undefined-behaviour sanitizers: contexts with every element kind, the
// coefficient-class and CPML table builders, the oblique-wire tables, tile
// lists, batch packing, and the documented error paths.  Prints "ok" and
// exits 0 when every call returned what it should.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fdtd.h"

static int fails = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("expectation failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

static fdtd_ctx* grid(int nx, int ny, int nz, int npml, int steps, bool debye, bool owire) {
  fdtd_params p;
  fdtd_default_params(&p);
  p.nx = nx; p.ny = ny; p.nz = nz; p.dx = 0.25; p.npml = npml; p.max_steps = steps;
  fdtd_ctx* c = nullptr;
  EXPECT(fdtd_create(&p, nullptr, &c) == FDTD_OK);
  std::vector<uint8_t> cm((size_t)nx * ny * nz);
  for (size_t i = 0; i < cm.size(); ++i) cm[i] = (uint8_t)((i / 7) % 3);
  const fdtd_material mats[3] = {{1, 0, 1}, {10, 0.01, 1}, {4, 0.002, 2}};
  EXPECT(fdtd_set_materials(c, cm.data(), mats, 3) == FDTD_OK);
  if (debye) {
    const double tau[2] = {1e-9, 2e-8}, deps[6] = {0, 0, 3, 1, 2, 0.5};
    EXPECT(fdtd_set_debye(c, 2, tau, deps) == FDTD_OK);
  }
  std::vector<double> amps(steps, 1.0);
  EXPECT(fdtd_add_wire(c, 0, 2, ny / 2, nz / 2, nx - 4, 0.004) == FDTD_OK);
  EXPECT(fdtd_add_wire(c, 2, nx / 3, ny / 3, 1, nz - 3, 0.01) == FDTD_OK);
  EXPECT(fdtd_add_source(c, FDTD_SRC_CURRENT, 2, nx / 2, ny / 2 + 1, nz / 2, amps.data(), steps) == FDTD_OK);
  EXPECT(fdtd_add_lumped(c, FDTD_LUMPED_R, 1, nx / 2 + 1, 3, 4, 50.0) == FDTD_OK);
  EXPECT(fdtd_add_source_r(c, FDTD_SRC_VOLTAGE, 0, nx / 2, ny / 2 + 2, nz / 2 + 1, amps.data(), steps, 25.0) ==
         FDTD_OK);
  if (owire) {
    const double a[3] = {npml + 1.3, npml + 1.7, npml + 1.2};
    const double b[3] = {nx - npml - 2.5, ny - npml - 2.2, nz - npml - 2.1};
    int id = -1;
    EXPECT(fdtd_add_oblique_wire(c, a, b, 0.002, 1, amps.data(), steps, 2, &id) == FDTD_OK && id == 0);
    // a second wire from the first one's end, joined there
    const double e[3] = {npml + 1.6, ny - npml - 2.4, nz - npml - 2.6};
    EXPECT(fdtd_add_oblique_wire(c, b, e, 0.004, -1, nullptr, 0, -1, &id) == FDTD_OK && id == 1);
    const int ids[2] = {0, 1}, ends[2] = {1, 0}, bad[2] = {0, 7};
    EXPECT(fdtd_join_oblique_wires(c, 1, ids, ends) == FDTD_EINVAL);
    EXPECT(fdtd_join_oblique_wires(c, 2, bad, ends) == FDTD_EINVAL);
    EXPECT(fdtd_join_oblique_wires(c, 2, ids, ends) == FDTD_OK);
    EXPECT(fdtd_join_oblique_wires(c, 2, ids, ends) == FDTD_EINVAL);   // already joined
  }
  int pid = -1;
  EXPECT(fdtd_add_probe(c, FDTD_PR_E, 2, nx / 2, ny / 2 + 1, nz / 2 + 1, 1, &pid) == FDTD_OK);
  EXPECT(fdtd_add_probe(c, FDTD_PR_VLINE, 0, 1, ny / 2 + 2, nz / 2, nx - 3, &pid) == FDTD_OK);
  EXPECT(fdtd_add_probe(c, FDTD_PR_ILOOP, 2, nx / 2, ny / 2 + 1, nz / 2, 1, &pid) == FDTD_OK);
  return c;
}

int main() {
  fdtd_params p;
  fdtd_default_params(&p);
  fdtd_ctx* c = nullptr;
  EXPECT(fdtd_create(&p, nullptr, &c) == FDTD_EINVAL);     // sizes left at zero
  p.nx = p.ny = p.nz = 8; p.dx = 0.5; p.dt = 1.0;
  EXPECT(fdtd_create(&p, nullptr, &c) == FDTD_EUNSTABLE);  // dt above Courant

  for (int npml : {0, 3}) {
    for (int debye = 0; debye < 2; ++debye) {
      fdtd_ctx* g = grid(23, 17, 15, npml, 30, debye, !debye);
      EXPECT(fdtd_add_wire(g, 5, 1, 1, 1, 2, 0.004) == FDTD_EINVAL);
      EXPECT(fdtd_add_probe(g, FDTD_PR_VLINE, 0, 1, 1, 1, 400, nullptr) == FDTD_ERANGE);
      EXPECT(fdtd_finalize(g) == FDTD_OK);
      EXPECT(fdtd_finalize(g) == FDTD_OK);                   // idempotent
      EXPECT(fdtd_workspace_bytes(g) > 0);
      EXPECT(fdtd_num_classes(g) > 0);
      EXPECT(fdtd_algorithmic_bytes_per_step(g) > 0);
      EXPECT(fdtd_add_wire(g, 0, 2, 2, 2, 2, 0.004) == FDTD_ESTATE);
      EXPECT(fdtd_set_kernel(g, FDTD_KERNEL_TB2, 8, 20) == FDTD_OK);
      EXPECT(fdtd_set_kernel(g, 9, 0, 0) == FDTD_EINVAL);
      EXPECT(fdtd_step(g, 1) == FDTD_ESTATE);                // no workspace bound
      double out[4];
      int nw = 0;
      EXPECT(fdtd_probe(g, 0, out, 4, &nw) != FDTD_OK);
      fdtd_destroy(g);
    }
  }
  // a source on a wire edge is refused when the tables are built
  fdtd_ctx* w = grid(20, 16, 14, 2, 10, false, false);
  std::vector<double> amps(10, 1.0);
  EXPECT(fdtd_add_source(w, FDTD_SRC_CURRENT, 0, 3, 8, 7, amps.data(), 10) == FDTD_OK);
  EXPECT(fdtd_finalize(w) == FDTD_ERANGE);
  fdtd_destroy(w);
  // the static binding refuses a grid beyond its array on the host
  fdtd_default_params(&p);
  p.nx = p.ny = p.nz = 168; p.dx = 0.5; p.max_steps = 4;
  EXPECT(fdtd_create(&p, nullptr, &c) == FDTD_OK);
  EXPECT(fdtd_bind_static(c) == FDTD_ENOMEM);
  fdtd_destroy(c);
  // batch packing of uneven grids with a CPML
  std::vector<fdtd_ctx*> gs;
  for (int q = 0; q < 4; ++q) gs.push_back(grid(24 + 5 * q, 20 + 3 * q, 18 + q, 4, 20, false, false));
  fdtd_batch* b = nullptr;
  EXPECT(fdtd_batch_pack(gs.data(), (int)gs.size(), nullptr, &b) == FDTD_OK);
  EXPECT(fdtd_batch_workspace_bytes(b) > 0);
  EXPECT(fdtd_batch_cells(b) > 0);
  EXPECT(fdtd_batch_set_kernel(b, 60, 8, 32, 4) == FDTD_OK);
  EXPECT(fdtd_batch_set_kernel(b, 48, 8, 32, 0) == FDTD_EINVAL);
  EXPECT(fdtd_batch_run(b, 1) == FDTD_ESTATE);
  fdtd_batch_destroy(b);
  for (fdtd_ctx* g : gs) fdtd_destroy(g);
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
