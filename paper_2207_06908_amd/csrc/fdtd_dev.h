// fdtd_dev.h -- device-side views of one grid, shared by the host runtime and
// the HIP kernels of this library.
#pragma once
#include <stdint.h>
#include <string>

namespace mi355fdtd {

// Coefficients of one class: the 9 numbers a node needs to update the six
// components it owns (Ex..Hz at the node's Yee positions).  The K_CA* slots
// hold ca - 1:
//   E_a^{n+1} = E_a^n + ((ca_a - 1) E_a^n + cb_a (difference of H))  [cb = Cb / dx]
//   H_a^{n+1/2} = H_a^{n-1/2} + db_a (difference of E)                [db = Db / dx]
enum { K_CAX = 0, K_CBX, K_CAY, K_CBY, K_CAZ, K_CBZ, K_DBX, K_DBY, K_DBZ, K_NCOEF };

// CPML profile table of one axis: 6 rows of 2*npml entries, indexed by the
// slab-local position l (l < npml: low slab, position l; l >= npml: high
// slab, position n - 2 npml + l).  Rows: b - 1, c, 1/kappa at the integer
// (E) position, then b - 1, c, 1/kappa at the half-integer (H) position.
enum { P_BE = 0, P_CE, P_IKE, P_BH, P_CH, P_IKH, P_NROW };

// Class table rows are padded to K_STRIDE values so a row loads as 3 x 4-wide.
enum { K_STRIDE = 12 };

// Device view of one grid for one launch.  Input and output pointers are
// resolved on the host (the in-place split variant passes the same set for
// both), so kernels index them only with compile-time constants.
template <typename T>
struct GridView {
  int nx, ny, nz, npml;
  long long sxy;                 // nx * ny
  long long ncell;               // nx * ny * nz
  int ncls;                      // number of coefficient classes
  int pad0;
  const T* fi[6];                // fields read  (E^n, H^{n-1/2}), components Ex..Hz
  T* fo[6];                      // fields written (E^{n+1}, H^{n+1/2})
  // CPML state of axis u: 4 arrays of pel[u] values each, starting at
  // pib[u] (input set) / pob[u] (output set), ordered [kind][component] with
  // kind 0 = E-type, 1 = H-type and component 0 the one along axis+1,
  // component 1 along axis+2.
  const T* pib[3];
  T* pob[3];
  unsigned pel[3];
  int pad2;
  const T* zpl;                  // nx * ny zeros: E of the planes outside [0, nz)
  const void* cls;               // class id per node (uint8 or uint16)
  const T* ctab;                 // [ncls][K_STRIDE]
  const T* prof[3];              // per axis [P_NROW][2*npml]
  // sources: E[src_comp][src_idx] -= src_amp[s * max_steps + n] after the
  // update; the list is grouped by column (x + nx*y), a node's own sources in
  // the order they were added, and src_first[column] is the column's run,
  // first | count << 20 (-1: none)
  int n_src;
  int max_steps;
  const int* src_comp;
  const long long* src_idx;
  const T* src_amp;
  const int* src_first;          // [nx * ny]
  const int* src_kr;             // [nx * ny]: planes of a column's sources, kmin | kmax << 16
  // probes: value p = sum over terms t in [pr_off[p], pr_off[p+1]) of
  // term_w[t] * field[term_comp[t]][term_idx[t]]
  int n_probe;
  int pad1;
  const int* pr_off;
  const int* term_comp;
  const long long* term_idx;
  const double* term_w;
  double* pr_out;                // [n_probe][max_steps]
  // step counter in device memory for launches replayed from a captured
  // graph: a kernel's step is *dstep plus its step argument (nullptr: the
  // argument alone)
  const int* dstep;
};

// Debye media (auxiliary differential equation): per E component a and
// pole p the polarisation current J (one array of ncell values each,
// j[a * 4 + p]; poles p >= npole point at pole npole - 1's array, which the
// kernels read but neither use nor write), per class and component the pole
// factors dtab[(class * 3 + a) * 8 + 2 p] = beta_p and [.. + 1] = gam_p,
// a per-class flag (any pole term), and the decay factors kp.  The update:
//   E^{n+1} = Ca E^n + Cb curl H - sources - sum_p gam_p J_p^n,
//   J_p^{n+1} = kp_p J_p^n + beta_p (E^{n+1} - E^n).
enum { D_MAXPOLE = 4, D_STRIDE = 3 * 2 * D_MAXPOLE };
template <typename T>
struct DebyeView {
  T* j[3 * D_MAXPOLE];
  const T* dtab;                 // [ncls][3][D_MAXPOLE][2]
  const unsigned char* dflag;    // [ncls]
  T kp[D_MAXPOLE];
  int npole;
};

}  // namespace mi355fdtd

namespace mi355fdtd {

// Oblique thin wires.  Wire w has nseg segments starting at seg0 in the
// segment arrays and nseg + 1 end-point charges starting at seg0 + w.  A
// segment samples E through its gather terms (the charge-conserving edge
// weights of its displacement) and feeds the same edges back: every edge a
// wire touches is a source of the grid (row wsrc[e] of the source list)
// whose amplitude, (Cb / dx) sum_t j_w I_seg, the wire kernels write for each
// step before the field pass applies it.
struct OWireParam {
  int seg0, nseg, src, rec;   // first segment, count, driven and recorded segment (-1: none)
  double dtL;                 // dt / L'
  double invCdl;              // 1 / (C' dl)
  double dtdl;                // dt / dl (interior end points; twice that at the two ends)
  double pad;
};
struct OWireView {
  int n_wire, max_steps, n_edge, max_seg;  // max_seg: segments of the longest wire
  const OWireParam* par;
  const int* seg_off;         // [total segments + 1]: gather terms of each segment
  const long long* g_key;     // E component << 40 | node index of a gather term
  const double* g_w;          // its weight: E_t = sum g_w E
  const long long* e_key;     // [n_edge] E edges the wires inject into (component << 40 | node)
  const int* e_off;           // [n_edge + 1]: injection terms of each edge
  const int* j_seg;           // segment of an injection term (increasing within an edge)
  const double* j_w;          // its weight: E -= (Cb / dx) sum j_w I_seg
  const double* amp;          // [n_wire][max_steps] driven-segment current (A)
  double* cur;                // segment currents (A)
  double* q;                  // end-point charges per unit length (C/m)
  double* rec;                // [n_wire][max_steps] recorded segment current
  const int* wsrc;            // [n_edge] source-list row of each touched edge
  const int* g_edge;          // per gather term: its edge's index in e_key
  double* e1;                 // [n_edge] E^{n+1} at the touched edges (two-step passes)
  // junctions: members jn_off[J] .. jn_off[J+1] of junction J, each the
  // index of its end node in q, its half segment (m) and its C' (F/m)
  int n_junc;
  const int* jn_off;
  const int* jn_q;
  const double* jn_a;
  const double* jn_c;
};

// Kernel launchers (fdtd_kernels.hip).  `view` points to a GridView<float>
// (prec 32) or GridView<double> (prec 64) whose in/out pointers are already
// resolved: the split variant (1) updates in place (in == out), the fused
// variant (2) reads one set and writes the other, the two-step variant (3)
// advances two steps from the input set to the output set.  `step` selects
// the (first) source sample.  Returns 0 or a hipError_t value.
int launch_step(int prec, const void* view, int cls16, int variant, int step, int tile_y, int tile_z,
                void* stream);
// Split step (H then E, in place) of a grid with Debye poles: `dview` is a
// DebyeView<float> or DebyeView<double>.
// Oblique wires, before the field pass.  launch_owire_iq: the segment
// currents of step `step` from the input E (from_e1 = 0) or from the edge
// values of launch_owire_e1 (from_e1 = 1), then the charges; the record.
// launch_owire_amp: the touched edges' source amplitudes of step `step` from
// the current segment currents.  launch_owire_e1: E^{step+1} at the touched
// edges, recomputed from the input set (its sources of `step` included),
// for the second step of a two-step pass.
int launch_owire_iq(int prec, const void* view, const OWireView* ow, int step, int from_e1, void* stream);
int launch_owire_amp(int prec, const void* view, int cls16, const OWireView* ow, int step, void* stream);
int launch_owire_e1(int prec, const void* view, int cls16, const OWireView* ow, int step, void* stream);
int launch_step_debye(int prec, const void* view, const void* dview, int cls16, int step, void* stream);
// Fused one-step pass (reads one field set, writes the other) of a grid with
// Debye poles (fdtd_debye.hip): over the 4-group tile list `tiles` / counts
// (as for launch_lists_step, variant 2, 8-row tiles; groups 1-3 on
// `stream2`) or, with tiles == nullptr, over 64 x 8 tiles of tile_z planes.
int launch_fused_debye(int prec, const void* view, const void* dview, int cls16, int step, int tile_z,
                       const void* tiles, const int* counts, void* stream, void* stream2);

// Fused (variant 2) or two-step (variant 3) pass of one grid over a tile
// list: `tiles` is a device array of int4 in 4 groups of counts[q] tiles, by
// the CPML slabs a tile reaches (halo included): 0 neither x nor y slabs, 1 x
// slabs only, 2 y slabs only, 3 both.  Every group carries z CPML code.
//   variant 2: (i0, j0, k0, k1); 32 x tile_y tiles in groups 1 and 3,
//              64 x tile_y in groups 0 and 2;
//   variant 3: (i0 | iw << 16, j0 | jh << 16, k0, k1) with iw <= 60,
//              jh <= tile_y.
// Group 0 runs on `stream`, groups 1-3 on `stream2` (the caller orders the
// two streams around the call; they write disjoint tiles).  counts[4] tiles
// after group 3 (fused: 32 x tile_y) read an oblique wire's source
// amplitudes: they run last on `stream2`, after it waits for the event
// `ev_src` (nullptr: no wait) that follows the wire kernels; in variant 3 the
// first counts[5] of them are clear of the x and y slabs and run as z-only
// tiles.  Variant 3 also records the probes of `step` on `stream2`, after
// that wait.
int launch_lists_step(int prec, const void* view, int cls16, int variant, int step, int tile_y, const void* tiles,
                      const int* counts, void* stream, void* stream2, void* ev_src);
// Record the probes of step `step` from the view's output set.
int launch_probes(int prec, const void* view, int step, void* stream);

// After a two-step pass (variant 3) from view.fi to view.fo: record the
// probes of steps `step` (recomputed from the input set; only if `first`)
// and `step` + 1.  A two-step pass over tile lists records `step` itself
// (launch_lists_step), so the caller passes first = 0 after it.
int launch_probes2(int prec, const void* view, int cls16, int step, int first, void* stream);

// Batched step over a tile list.  `views` is a device array of GridView (one
// per grid, already resolved for this step's field-set parity), `tiles` a
// device array of int4 (grid, i0, j0, k0 | kz << 16).  The step index is
// *d_step + offset.  Tile shapes (tx, ty): (32, 8), (32, 16), (64, 8).
int launch_batch_step(int prec, int cls16, int pml, const void* views, const void* tiles, int n_tiles, int tx,
                      int ty, const int* d_step, int offset, void* stream);
// Batched probes: `plist` is a device array of int2 (grid, probe id).
int launch_batch_probes(int prec, const void* views, const void* plist, int n, const int* d_step, int offset,
                        void* stream);
// Batched two-step pass: `views` as for launch_batch_step (input set = the
// pass's input), `tiles` a device array of int4 (grid, i0 | iw << 16,
// j0 | jh << 16, k0 | kz << 16) in 4 CPML groups of counts[q] tiles (as for
// launch_lists_step), 60 x 8 tiles; then the probes of both steps for the
// (grid, probe) pairs of `plist`.  Steps *d_step + offset and + 1.  With a
// second stream (and two events), group 1 runs on it beside the others,
// forked from and joined back to `stream` before the probes.
int launch_batch_pass_tb2(int prec, int cls16, const void* views, const void* tiles, const int* counts,
                          const void* plist, int n_probes, const int* d_step, int offset, void* stream,
                          void* stream2, void* ev_fork, void* ev_join);
// Batched two-step pass as persistent launches (k_tb2_batch_q), one per code
// path: path A (the x-slab instantiation) over tiles_a with blocks_a blocks
// on `stream`, path B (the all-axes one) over tiles_b with blocks_b blocks
// on `stream2` (forked and joined with the events when both have tiles; a
// path with 0 blocks is skipped).  Tiles are int4 (grid | group << 24,
// i0 | iw << 16, j0 | jh << 16, k0 | kz << 16), grid by grid, in 8 runs
// [runs.start[x], runs.start[x + 1]), one per XCD; `ctr` is 16 device ints
// (A's 8, then B's; reset on the stream before the launches).  Then the
// probes of both steps, as for launch_batch_pass_tb2.
struct QRuns {
  int start[9];
};
// Blocks of k_tb2_batch_q for path axp (5: A, 7: B) that fit on the device
// at once (0 on error).
int batch_queue_blocks(int prec, int cls16, int axp);
int launch_batch_pass_queue(int prec, int cls16, const void* views, const void* tiles_a, const QRuns* runs_a,
                            int blocks_a, const void* tiles_b, const QRuns* runs_b, int blocks_b, int* ctr,
                            const void* plist, int n_probes, const int* d_step, int offset, void* stream,
                            void* stream2, void* ev_fork, void* ev_join);
// *d += v on the stream (advances the device step counter).
int launch_add(int* d, int v, void* stream);
// *d = v on the stream.
int launch_set(int* d, int v, void* stream);
}  // namespace mi355fdtd

// Host-side hooks between fdtd_host.cpp and fdtd_static.hip: record an
// error message on a context and return its code; drop a context's claim on
// the static workspace of any device (called by fdtd_destroy).
struct fdtd_ctx;
int fdtd_fail_code(fdtd_ctx* c, int code, const std::string& msg);
void fdtd_static_release(const fdtd_ctx* c);
