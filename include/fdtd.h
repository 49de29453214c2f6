/*
 * fdtd.h -- C ABI of the MI355X (gfx950) Yee FDTD library.
 *
 * The library advances Maxwell's curl equations (Kuklin, "elecode",
 * Section 2.1, eq. 1) on a uniform staggered Yee grid: the E update of eq. 4
 * and the H update of eq. 5, with the other components by cyclic permutation,
 * per-cell eps, sigma and mu (eqs. 2-3), an ideal lumped current source
 * (Section 2.1), a convolutional PML backed by perfect-conductor walls
 * (Section 2.2) and thin wires along grid edges by modification of the
 * assigned material parameters (Section 2.3).
 *
 * Geometry.  Node (i, j, k) is the point (i, j, k) dx.  Cell (i, j, k) spans
 * [i, i+1] x [j, j+1] x [k, k+1] (units of dx).  An edge is (axis, start node)
 * and spans node -> node + e_axis.  The component stored at node (i, j, k) is
 * Ex at (i+1/2, j, k), Ey at (i, j+1/2, k), Ez at (i, j, k+1/2),
 * Hx at (i, j+1/2, k+1/2), Hy at (i+1/2, j, k+1/2), Hz at (i+1/2, j+1/2, k).
 * Host arrays are x fastest: element (i, j, k) at i + nx (j + ny k).
 *
 * Time levels.  The state entering step n is (E^n, H^{n-1/2}), all zero at
 * creation.  Step n updates H to n+1/2, then E to n+1 including the source
 * current sampled at (n+1/2) dt, then records the probes: E and line-voltage
 * probes hold E^{n+1}, loop-current probes hold H^{n+1/2}.
 *
 * Ownership.  The caller owns every host array it passes (copied during the
 * call) and the device workspace (allocated by the caller, e.g. as a PyTorch
 * tensor, and bound by pointer).  The library never allocates device memory
 * on the stepping path; it places its fields, tables and probe records inside
 * the workspace and owns their contents.  All device work is issued on the
 * stream given at creation (NULL = the default stream).
 *
 * Errors.  Every int-returning call returns FDTD_OK (0) or a negative FDTD_E*
 * code and records a message for fdtd_last_error.  No call aborts or exits.
 * Set-up calls validate on the host before any HIP call, so every error path
 * except FDTD_EDEVICE is reachable without a GPU.  A context is not
 * thread-safe; distinct contexts are independent.
 */
#ifndef MI355_FDTD_H
#define MI355_FDTD_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  FDTD_OK = 0,
  FDTD_EINVAL = -1,     /* null pointer, bad axis / kind / count, radius not in (0, dx/2) */
  FDTD_ERANGE = -2,     /* index outside the grid, source on a wall or wire edge, beyond max_steps */
  FDTD_ESTATE = -3,     /* set-up call after the workspace size was taken, step before binding */
  FDTD_EUNSTABLE = -4,  /* dt above the Courant limit, or literal eq. 4 loss with sigma dt / eps >= 2 */
  FDTD_ENOMEM = -5,     /* workspace smaller than fdtd_workspace_bytes, or misaligned */
  FDTD_EDEVICE = -6,    /* a HIP runtime call failed */
  FDTD_ENONFINITE = -7, /* NaN or Inf in an input array */
  FDTD_ECLASS = -8      /* more than 65535 distinct coefficient classes */
};
enum { FDTD_EX = 0, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ };
enum { FDTD_PR_E = 0, FDTD_PR_VLINE = 1, FDTD_PR_ILOOP = 2 };
enum { FDTD_LOSS_SEMI = 0, FDTD_LOSS_EXPLICIT = 1 };
enum { FDTD_SRC_CURRENT = 0, FDTD_SRC_VOLTAGE = 1 };
enum { FDTD_LUMPED_R = 0, FDTD_LUMPED_C = 1 };
/* Kernel variants for fdtd_set_kernel: two passes per step (H, then E), one
 * fused pass per step, or one temporally blocked pass per two steps (an odd
 * remaining step takes one fused pass).  FDTD_KERNEL_AUTO (the default) is
 * the two-step pass for grids with a CPML and the fused pass otherwise.  The
 * two-step pass needs 2 npml <= 128 (FP32) or 64 (FP64); thicker CPMLs take
 * the fused pass. */
enum { FDTD_KERNEL_AUTO = 0, FDTD_KERNEL_SPLIT = 1, FDTD_KERNEL_FUSED = 2, FDTD_KERNEL_TB2 = 3 };

typedef struct fdtd_ctx fdtd_ctx;
typedef struct { double eps_r, sigma, mu_r; } fdtd_material;

typedef struct {
  int nx, ny, nz;            /* cells along x, y, z (>= 2 each) */
  double dx;                 /* cubic cell size [m] */
  double dt;                 /* time step [s]; <= 0 selects 0.99 dx / (c0 sqrt(3)) */
  int npml;                  /* CPML cells on each of the six faces; 0 = bare PEC box */
  double pml_m;              /* grading order m of sigma and kappa (default 3) */
  double pml_sigma_factor;   /* sigma_max = factor * 0.8 (m + 1) / (eta0 dx) (default 1) */
  double pml_kappa_max;      /* default 1 */
  double pml_alpha_max;      /* [S/m], default 0 */
  double pml_ma;             /* grading order of alpha (default 1) */
  int loss_mode;             /* FDTD_LOSS_SEMI (default) or FDTD_LOSS_EXPLICIT (eq. 4 as printed) */
  double wire_r0_factor;     /* equivalent radius of a bare wire edge / dx, in (0, 1); default exp(-pi/2) */
  int max_steps;             /* capacity of the probe records (total steps allowed) */
  int precision;             /* 32 (default) or 64: floating-point type of fields and arithmetic */
} fdtd_params;

/* Fill *p with the defaults above (grid size and dx left at zero). */
void fdtd_default_params(fdtd_params* p);

/* Validate p and create a host-side context for one grid (the uniform
 * staggered Yee grid of Section 2.1, eqs. 4-5, with the CPML of Section 2.2
 * when npml > 0).  hip_stream is a hipStream_t or NULL.  Errors: EINVAL (bad sizes, npml leaves no interior, bad precision or
 * loss mode), EUNSTABLE (dt above the Courant limit). */
int fdtd_create(const fdtd_params* p, void* hip_stream, fdtd_ctx** out);

/* Per-cell material ids (nx*ny*nz bytes, x fastest) into a table of n_mat
 * materials (eps_r > 0, sigma >= 0, mu_r > 0).  Without this call every cell
 * is vacuum.  Edge eps and sigma are the arithmetic mean over the cells
 * sharing the edge; face mu is the harmonic mean of the two cells sharing the
 * face.  Errors: EINVAL, ERANGE (id >= n_mat), ENONFINITE, ESTATE. */
int fdtd_set_materials(fdtd_ctx* c, const uint8_t* cell_mat, const fdtd_material* tab, int n_mat);

/* Debye media (Section 2.4, auxiliary differential equation), after
 * fdtd_set_materials (which drops earlier poles): n_poles in 1..4 time
 * constants tau [s] shared by the grid, and for each material m of that
 * table the pole increments d_eps[m * n_poles + p] (dimensionless, >= 0; 0
 * for non-dispersive materials).  A material's eps_r is then its eps_inf and
 * its sigma the static conductivity.  Edges average the increments like eps;
 * the radial edges of a thin wire scale them by the wire's factor like eps.
 * Each pole adds a polarisation current per E component,
 *   tau_p dJ_p/dt + J_p = eps0 d_eps_p dE/dt,
 * taken at n + 1/2 with the trapezoidal rule, like sigma E; J_p lives in the
 * workspace (3 n_poles extra arrays of nx*ny*nz values).  Such a grid runs
 * the split pass, or the fused pass when fdtd_set_kernel asks for it (8-row
 * tiles whatever tile_y asks; a two-step request takes the split pass), and
 * cannot join a batch.
 * Needs the semi-implicit loss form.  Errors: EINVAL, ENONFINITE, ESTATE. */
int fdtd_set_debye(fdtd_ctx* c, int n_poles, const double* tau, const double* d_eps);

/* Perfect-conductor thin wire of the given radius along +axis from node
 * (i, j, k) over n_cells edges (Section 2.3).  The wire's edges are held at
 * zero; eps and sigma of the radial edges at its nodes are multiplied by
 * m = ln(1 / wire_r0_factor) / ln(dx / radius); mu of the H circulating
 * around its segments (and the one segment past each end) and of the H
 * parallel to it around its nodes is divided by m.  Errors: EINVAL, ERANGE,
 * ESTATE. */
int fdtd_add_wire(fdtd_ctx* c, int axis, int i, int j, int k, int n_cells, double radius);

/* Ideal current source on the edge (axis, i, j, k): after the edge's update,
 * E -= Cb * I / dx^2 with Cb the edge's curl coefficient and I = amps[n] at
 * step n (amperes at (n+1/2) dt, positive toward +axis; 0 beyond n_samples).
 * The edge must be one the update touches (not on a wall) and not a wire
 * edge (checked when stepping starts).  Errors: EINVAL, ERANGE, ENONFINITE,
 * ESTATE. */
int fdtd_add_source(fdtd_ctx* c, int kind, int axis, int i, int j, int k,
                    const double* amps, int n_samples);

/* Oblique thin wire (Section 2.3: the arbitrarily located wire model the
 * paper lists beside the axis-aligned ones).  A straight wire from a to b
 * (x, y, z in cells, node (0,0,0) at the origin; both ends at least one cell
 * clear of the CPML and the walls; at least one cell long) of radius
 * 0 < radius < wire_r0_factor dx.  It gets floor(length) segments of equal
 * length dl with currents I_k at the segment midpoints and charges per unit
 * length q_k at their ends (open ends), stepped by the telegraph equations
 *   L' dI_k/dt = E_t(mid_k) - (q_{k+1} - q_k) / (C' dl),  dq_k/dt = -dI/dl,
 * L' = mu0 ln(r0/radius) / (2 pi), C' = 2 pi eps0 / ln(r0/radius),
 * r0 = wire_r0_factor dx.  The coupling conserves charge: the grid holds
 * the wire's node charges with cloud-in-cell weights, segment k's current
 * enters the E edges around it as the fluxes of Esirkepov's density
 * decomposition for the move from node k to node k+1 (E -= Cb J after the E
 * update, each touched edge summing its terms in a fixed order), and E_t,k
 * is the same-weighted sum of those edges' E over the segment length.
 * src_seg >= 0 drives that segment's current with amps[n] (A, at
 * (n + 1/2) dt; 0 after the last sample; n_amps may be 0); rec_seg >= 0
 * records that segment's current every step.  Every pass variant takes
 * oblique wires (in the two-step pass the touched edges are sources whose
 * amplitudes the wire kernels write before each pass; all variants give the
 * same bits).  Grids with oblique wires cannot take Debye media
 * (FDTD_EINVAL either way round) and cannot join a batch.  id (may be NULL)
 * receives the wire's index.
 * FDTD_ERANGE for an end point out of range or a segment index outside
 * [-1, n_seg), FDTD_ENONFINITE for a non-finite end point or sample,
 * FDTD_ESTATE after the workspace size was taken. */
int fdtd_add_oblique_wire(fdtd_ctx* ctx, const double* a, const double* b, double radius, int src_seg,
                          const double* amps, int n_amps, int rec_seg, int* id);

/* Junction of oblique wires (the multiwire junctions of the oblique-wire
 * formalism Section 2.3 cites): the n >= 2 wire ends ids[m], ends[m] (0: the
 * wire's start a, 1: its end b), which must meet at one point (within 1e-6
 * cells), become one node.  Its charge Q = sum_m q_m dl_m / 2 changes by
 * the currents that flow into the point, and the members share one
 * potential: q_m = C'_m Q / sum_m C'_m dl_m / 2.  A wire cut at one of its
 * nodes and rejoined there is the uncut wire.  FDTD_EINVAL for n < 2, a bad
 * id or end, an end listed twice or already in a junction, or ends that do
 * not meet; FDTD_ESTATE after the workspace size was taken. */
int fdtd_join_oblique_wires(fdtd_ctx* ctx, int n, const int* ids, const int* ends);

/* State of oblique wire id: segment currents (n_seg values, A), end-point
 * charges per unit length (n_seg + 1, C/m) and the recorded current
 * (min(steps done, n_rec_max) values) into host arrays; any of cur, q, rec
 * may be NULL (then nothing is copied for it, and with all three NULL only
 * n_seg is set, also before a workspace is bound).  Waits for the
 * library's stream.  n_written (may be NULL) receives the record length,
 * 0 without rec or a recorded segment. */
int fdtd_oblique_wire_read(fdtd_ctx* ctx, int id, double* cur, double* q, double* rec, int n_rec_max, int* n_seg,
                           int* n_written);

/* Lumped resistor (kind FDTD_LUMPED_R, value R [ohm] > 0) or capacitor
 * (FDTD_LUMPED_C, value C [F] > 0) across the E edge (axis, i, j, k)
 * (Section 2.1, lumped circuit elements): the edge's conductivity grows by
 * 1 / (R dx), its permittivity by C / dx, after any thin-wire change.
 * Elements on one edge add up.  Same edge rules as a source.  Errors:
 * EINVAL, ERANGE, ENONFINITE, ESTATE. */
int fdtd_add_lumped(fdtd_ctx* c, int kind, int axis, int i, int j, int k, double value);

/* Non-ideal source (Section 2.1), as its Norton equivalent: FDTD_SRC_CURRENT
 * is a current source (amps in A) with a shunt resistance r_internal [ohm]
 * (r_internal <= 0: ideal, as fdtd_add_source); FDTD_SRC_VOLTAGE is a voltage
 * source (amps in V, positive when the +axis end is the positive terminal)
 * with a series resistance r_internal > 0, i.e. the current V / r_internal
 * in parallel with r_internal.  Errors: as fdtd_add_source and
 * fdtd_add_lumped. */
int fdtd_add_source_r(fdtd_ctx* c, int kind, int axis, int i, int j, int k, const double* amps, int n_samples,
                      double r_internal);

/* Probe (recorded every step, FP64), the quantities the paper's model files
 * ask for with their output and calculate commands (Section 4.1): a field
 * component, a voltage as a line integral of E, a current as a loop
 * integral of H:
 *   FDTD_PR_E      value of the edge (axis, i, j, k) (n_cells = 1);
 *   FDTD_PR_VLINE  sum of E_axis dx over n_cells edges from node (i, j, k)
 *                  along +axis, i.e. phi(start) - phi(end);
 *   FDTD_PR_ILOOP  loop integral of H around the edge (axis, i, j, k),
 *                  right-handed about +axis (n_cells = 1).
 * Errors: EINVAL, ERANGE, ESTATE. */
int fdtd_add_probe(fdtd_ctx* c, int kind, int axis, int i, int j, int k, int n_cells, int* probe_id);

/* Freeze the set-up (later set-up calls return ESTATE) and build the
 * coefficient classes, CPML profiles, source and probe tables on the host.
 * Idempotent.  Errors: ERANGE (source on a wire edge), EUNSTABLE (literal
 * eq. 4 loss with sigma dt / eps >= 2), ECLASS. */
int fdtd_finalize(fdtd_ctx* c);

/* Device bytes the context needs (calls fdtd_finalize first).  Returns 0 on
 * error (see fdtd_last_error). */
size_t fdtd_workspace_bytes(fdtd_ctx* c);

/* Bind caller-owned device memory of at least fdtd_workspace_bytes bytes,
 * 256-byte aligned.  Uploads the tables and zeroes the fields on the stream.
 * Errors: ENOMEM, ESTATE, EDEVICE. */
int fdtd_bind_workspace(fdtd_ctx* c, void* dev_ptr, size_t bytes);

/* Allocation-free binding, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): instead of a caller-owned workspace, the context uses a static
 * device array of FDTD_STATIC_BYTES (64 MiB) that the library holds on each
 * GPU it runs on until the process ends -- enough for a 48^3 grid with all
 * its tables, or about a million cells in FP32.  It binds the array of the
 * current device (the context's stream must belong to it), then behaves as
 * fdtd_bind_workspace: tables uploaded, every field, CPML, wire state and
 * probe record zeroed, so nothing an earlier context left in the array
 * survives.  Only one live context per device may hold the array: binding a
 * second one returns FDTD_ESTATE until the first is destroyed (work of two
 * contexts on one array would race).  Calls no hipMalloc or hipFree.
 * Errors: ENOMEM (workspace larger than FDTD_STATIC_BYTES, checked before
 * any HIP call), ESTATE (already bound, or the array is held), EDEVICE, and
 * fdtd_finalize's errors. */
#define FDTD_STATIC_BYTES ((size_t)64 << 20)
int fdtd_bind_static(fdtd_ctx* c);

/* Select a kernel variant (FDTD_KERNEL_*) and tile parameters (0 = default:
 * 8 rows; 20 planes for the two-step pass, 32 otherwise): tile_y (rows per
 * tile) in {4, 8}, or 12 for FDTD_KERNEL_TB2; tile_z (planes per z chunk)
 * >= 0.  Grids with a CPML run the fused and two-step passes over tile
 * lists grouped by the CPML slabs each tile reaches; tile_z applies to the
 * tiles clear of the x and y slabs, the slab groups take chunks of
 * min(tile_z, 20) planes (two-step) or max(8, tile_z / 4) (fused).
 * Results do not depend on the choice (bitwise).  Errors: EINVAL. */
int fdtd_set_kernel(fdtd_ctx* c, int variant, int tile_y, int tile_z);

/* Graph replay: graph_steps (a multiple of 4; 0 = off, the default) steps
 * of launches are captured once into a HIP graph (per parity of the field
 * set they start from) and replayed for each run of that many steps, the
 * kernels taking the step from a counter in the workspace.  For small grids,
 * whose steps are short next to the launch overhead.  Results do not depend
 * on it (bitwise).  While timing is enabled, a replay is timed whole, its
 * probe kernels included.  Errors: EINVAL. */
int fdtd_set_graph(fdtd_ctx* c, int graph_steps);

/* Advance n_steps steps of the leapfrog scheme (Section 2.1: the H update
 * of eq. 5, then the E update of eq. 4 with the sources, then the probes),
 * asynchronously on the stream.  Errors: ESTATE (not
 * bound), ERANGE (beyond max_steps), EDEVICE. */
int fdtd_step(fdtd_ctx* c, int n_steps);

/* Copy probe_id's record (one double per completed step, at most n_max) to
 * out; synchronises the stream.  Errors: EINVAL, ESTATE, EDEVICE,
 * ENONFINITE (the record holds NaN or Inf; the data is still copied). */
int fdtd_probe(fdtd_ctx* c, int probe_id, double* out, int n_max, int* n_written);

/* Whole-component host copies (nx*ny*nz doubles, x fastest; comp FDTD_EX ..
 * FDTD_HZ).  set_field zeroes perfect-conductor edges (walls, wires).
 * Both synchronise the stream.  Errors: EINVAL, ESTATE, EDEVICE. */
int fdtd_set_field(fdtd_ctx* c, int comp, const double* host);
int fdtd_get_field(fdtd_ctx* c, int comp, double* host);

/* Diagnostics: the time step in use, steps taken, coefficient classes, and
 * the bytes one step moves at the algorithmic minimum (fields read and
 * written once, class ids, CPML state) -- the roofline numerator. */
double fdtd_dt(const fdtd_ctx* c);
long long fdtd_steps_done(const fdtd_ctx* c);
int fdtd_num_classes(const fdtd_ctx* c);
double fdtd_algorithmic_bytes_per_step(const fdtd_ctx* c);

/* Kernel timing for roofline measurement: while enabled, fdtd_step records a
 * HIP event pair on the context's stream around the update kernels of every
 * step (not around the probe-recording kernel).  fdtd_kernel_time
 * synchronises, returns the summed event time and the number of timed steps
 * since the last call, and resets both.  Errors: EINVAL, EDEVICE. */
int fdtd_timing(fdtd_ctx* c, int enable);
int fdtd_kernel_time(fdtd_ctx* c, double* total_ms, long long* n_steps);

const char* fdtd_last_error(const fdtd_ctx* c);
void fdtd_destroy(fdtd_ctx* c);

/* ---------------------------------------------------------------------------
 * Batched engine: many independent grids (e.g. a parameter sweep of small,
 * uneven electrode grids) stepped together, one kernel launch per step (or
 * two persistent launches per two-step pass, one per code path) over tile
 * lists that span every grid, optionally replayed from a captured HIP
 * graph.  Each grid's results are bit-identical to running it alone.
 * ------------------------------------------------------------------------- */
typedef struct fdtd_batch fdtd_batch;

/* Pack n fully set-up contexts (finalized here if needed, not yet bound to a
 * workspace; same precision, all with or all without CPML, all with 1-byte
 * or all with 2-byte class ids).  The batch borrows the contexts: destroy
 * the batch before them.  After binding, fdtd_probe / fdtd_get_field on a
 * member context read its part of the batch workspace.  Errors: EINVAL,
 * ESTATE (a context already bound), and fdtd_finalize's errors. */
int fdtd_batch_pack(fdtd_ctx* const* grids, int n, void* hip_stream, fdtd_batch** out);
size_t fdtd_batch_workspace_bytes(const fdtd_batch* b);
/* Caller-owned device memory, 256-byte aligned.  Errors: ENOMEM, ESTATE, EDEVICE. */
int fdtd_batch_bind_workspace(fdtd_batch* b, void* dev_ptr, size_t bytes);
/* Tile shape (tile_x, tile_y) in {(32, 8), (32, 16), (64, 8)}, z-chunk
 * tile_z in [8, 4096]; graph_steps (even, 0 = off): steps captured in one
 * HIP graph and replayed.  (60, 8) selects two-step passes (two time steps
 * per launch sequence, tiles grouped by the CPML slabs they reach, the
 * x-slab group on a second stream of the library's beside the others) with
 * tile_z in [16, 4096] and graph_steps a multiple of 4 (every grid with
 * 2 npml <= 128 in FP32, 64 in FP64); an odd step count ends with one
 * single-step launch.  Results do not depend on the choice.
 * Default (32, 8, 32, 0).  Errors: EINVAL. */
int fdtd_batch_set_kernel(fdtd_batch* b, int tile_x, int tile_y, int tile_z, int graph_steps);
/* Two-step passes only: on = 1 (the default) runs each pass as persistent
 * launches whose blocks take tiles from work queues: one launch for the
 * tiles clear of the y slabs (the x-slab code path), one on the second
 * stream for the rest (the all-axes path; every tile in FP64), each XCD
 * starting on its own run of a queue's tiles, grid by grid.  on = 0
 * launches the CPML groups separately (the x-slab group on the second
 * stream).  Results do not depend on the choice.  Errors: EINVAL. */
int fdtd_batch_set_persistent(fdtd_batch* b, int on);
/* Advance every grid n_steps steps.  Errors: ESTATE, ERANGE (beyond the
 * smallest max_steps), EDEVICE. */
int fdtd_batch_run(fdtd_batch* b, int n_steps);
/* Samples of probe probe_id of member grid `grid` (its index in the packed
 * array), as fdtd_probe: syncs the stream, copies min(n_max, steps run)
 * FP64 samples to the caller's host buffer.  Errors: EINVAL (no such grid
 * or probe, null pointers), ESTATE (not bound), EDEVICE. */
int fdtd_batch_probe(fdtd_batch* b, int grid, int probe_id, double* out, int n_max, int* n_written);
/* Wall time of fdtd_batch_run calls made while timing is enabled (HIP
 * events on the stream); fdtd_batch_time returns and resets the totals. */
int fdtd_batch_timing(fdtd_batch* b, int enable);
int fdtd_batch_time(fdtd_batch* b, double* total_ms, long long* n_steps);
long long fdtd_batch_cells(const fdtd_batch* b);
double fdtd_batch_algorithmic_bytes_per_step(const fdtd_batch* b);
const char* fdtd_batch_last_error(const fdtd_batch* b);
void fdtd_batch_destroy(fdtd_batch* b);

#ifdef __cplusplus
}
#endif
#endif
