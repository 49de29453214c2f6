/*
 * orc.h -- FP64 CPU reference for the 3D Yee FDTD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with
 * the GPU library; the two are fed the same seeded inputs and nothing else.
 *
 * What it computes (Kuklin, "elecode", Section 2):
 *   - Maxwell's curl equations (eq. 1) in component form for E with a
 *     conducting medium (eq. 2) and for H (eq. 3);
 *   - their Yee leapfrog discretisation: the Ex update of eq. 4 and the Hx
 *     update of eq. 5, with the other four components by cyclic permutation;
 *   - lossy coefficients either in the literal form of eq. 4 or in the
 *     semi-implicit form the paper allows "for better accuracy" (Section 2.1);
 *   - an ideal lumped current source (Section 2.1, sources);
 *   - a convolutional PML (Section 2.2);
 *   - a thin wire along grid edges by modification of the assigned material
 *     parameters next to the wire (Section 2.3).
 * Readings of what the paper leaves open are stated at each function.
 *
 * All calls return 0 on success or a negative ORC_E* code; nothing aborts.
 * Field exchange layout: one array per component of nx*ny*nz doubles, x
 * fastest; entry (i,j,k) is the component stored at node (i,j,k) (e.g. Ex at
 * ((i+1/2)dx, j dx, k dx)).  Components on the upper walls (index nx, ny or
 * nz) are identically zero and are not part of the exchange.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_ESTATE = -3, ORC_EUNSTABLE = -4 };
enum { ORC_EX = 0, ORC_EY, ORC_EZ, ORC_HX, ORC_HY, ORC_HZ };
enum { ORC_PR_E = 0, ORC_PR_VLINE = 1, ORC_PR_ILOOP = 2 };
enum { ORC_LOSS_SEMI = 0, ORC_LOSS_EXPLICIT = 1 };
enum { ORC_SRC_CURRENT = 0, ORC_SRC_VOLTAGE = 1 };
enum { ORC_LUMPED_R = 0, ORC_LUMPED_C = 1 };

typedef struct orc_sim orc_sim;
typedef struct { double eps_r, sigma, mu_r; } orc_material;
typedef struct {
  int nx, ny, nz;
  double dx;                 /* uniform cubic cells [m] */
  double dt;                 /* <= 0 selects 0.99 of the 3D Courant limit */
  int npml;                  /* CPML thickness in cells on all six faces (0 = bare PEC box) */
  double pml_m, pml_sigma_factor, pml_kappa_max, pml_alpha_max, pml_ma;
  int loss_mode;             /* ORC_LOSS_SEMI or ORC_LOSS_EXPLICIT */
  double wire_r0_factor;     /* equivalent radius of a bare wire edge, in cells (exp(-pi/2) typical) */
  int max_steps;             /* capacity of the probe records */
} orc_params;

int  orc_create(const orc_params* p, orc_sim** out);
void orc_destroy(orc_sim* s);
int  orc_set_threads(int n);
int  orc_set_materials(orc_sim* s, const uint8_t* cell_mat, const orc_material* tab, int n_mat);
/* Debye media (Section 2.4), after orc_set_materials: n_poles (1..4) time
 * constants tau [s] shared by the grid and, per material of that table, the
 * pole increments d_eps[m * n_poles + p] (dimensionless, >= 0); the
 * material's eps_r is then eps_inf and its sigma the static conductivity.
 * Needs the semi-implicit loss form. */
int  orc_set_debye(orc_sim* s, int n_poles, const double* tau, const double* d_eps);
int  orc_add_wire(orc_sim* s, int axis, int i, int j, int k, int n_cells, double radius);
int  orc_add_source(orc_sim* s, int axis, int i, int j, int k, const double* amps, int n);
/* Lumped resistor (R [ohm]) or capacitor (C [F]) on an updated E edge:
 * sigma += 1 / (R dx), eps += C / dx on that edge. */
int  orc_add_lumped(orc_sim* s, int kind, int axis, int i, int j, int k, double value);
/* Non-ideal source: current source with shunt resistance r (r <= 0 ideal),
 * or voltage source [V] with series resistance r > 0 (Norton equivalent). */
int  orc_add_source_r(orc_sim* s, int kind, int axis, int i, int j, int k, const double* amps, int n, double r);
int  orc_add_probe(orc_sim* s, int kind, int axis, int i, int j, int k, int n_cells, int* id);
/* Oblique thin wire from a to b (cell units, node (0,0,0) at the origin,
 * at least one cell long, clear of the CPML and the walls by one cell),
 * radius < wire_r0_factor dx; src_seg >= 0 drives that segment's current
 * with amps (A, sampled at (n + 1/2) dt); rec_seg >= 0 records that
 * segment's current each step.  Not with Debye media. */
int  orc_add_oblique_wire(orc_sim* s, const double* a, const double* b, double radius, int src_seg,
                          const double* amps, int n_amps, int rec_seg, int* id);
/* Junction: the listed wire ends (ends[m] = 0: the wire's start a, 1: its
 * end b) meet at one point (within 1e-6 cells) and become one node: its
 * charge follows the currents flowing into it, and its members share one
 * potential q / C'.  Each wire end joins at most one junction; n >= 2. */
int  orc_join_oblique_wires(orc_sim* s, int n, const int* ids, const int* ends);
/* Segment currents (n_seg), end-point charges per unit length (n_seg + 1),
 * and the record (any pointer may be NULL). */
int  orc_oblique_wire_read(orc_sim* s, int id, double* cur, double* q, double* rec, int n_rec_max,
                           int* n_seg, int* n_written);
int  orc_step(orc_sim* s, int n_steps);
int  orc_probe(orc_sim* s, int id, double* out, int n_max, int* n_written);
int  orc_set_field(orc_sim* s, int comp, const double* v);
int  orc_get_field(orc_sim* s, int comp, double* v);
/* which = 0: Ca (E comps) or Db (H comps); which = 1: Cb (E comps). */
int  orc_get_coef(orc_sim* s, int comp, int which, double* v);
double orc_dt(const orc_sim* s);
const char* orc_last_error(const orc_sim* s);

#ifdef __cplusplus
}
#endif
#endif
