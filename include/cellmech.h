/*
 * cellmech: Mooney-Rivlin tetrahedral cell forces on AMD Instinct MI355X
 * (gfx950).  C ABI of the device library libcellmech.so.
 *
 * Method (Mueller et al., "A hyperelastic model for simulating cells in
 * flow", arXiv 2003.03130):
 *   For every tetrahedron with reference vertices x^1..x^4 and deformed
 *   vertices y^1..y^4 (vertex 4 is the local origin):
 *     J_ik = x_i^k - x_i^4, B = J^-1, V0 = |det J| / 6   (Jacobian paragraph,
 *                                                         computed once)
 *     F = D_s B with (D_s)_ik = y_i^k - y_i^4             (eq. displacement-
 *                                                         derivative: F = I + AB)
 *     C = F^T F, J = det F, I = tr(C) J^-2/3,
 *     K = (tr(C)^2 - tr(C^2)) / 2 J^-4/3                  (eqs. invariantJ/I/K)
 *     U = mu1/2 (I - 3) + mu2/2 (K - 3) + kappa/2 (J - 1)^2
 *                                                         (eq. strain-energy-
 *                                                          density:mr)
 *     mu1 = w mu, mu2 = (1 - w) mu                         (Sec. "Theory")
 *     f^a = -V0 dU/dy^a                                    (eq. elastic-force-
 *                                                          vertex-0, evaluated
 *                                                          with the chain rule
 *                                                          of eq. -vertex-1)
 *   The node force is the sum over the tetrahedra sharing the node and the
 *   cell energy is E = sum V0 U, so f = -grad_y E.
 *   For J <= 0 (an inverted tetrahedron) J^-1/3 is the reciprocal of the
 *   sign-preserving real cube root; such tetrahedra are counted, not rejected.
 *
 * Conventions shared by every call:
 *   - A handle holds one or more cells ("batch").  Node and tetrahedron
 *     arrays of all cells are concatenated; node_off / tet_off are CSR
 *     offsets with n_cells + 1 entries.
 *   - Node arrays on the device are structure-of-arrays float32:
 *     x-components of all nodes, then y-components, then z-components
 *     (3 * n_nodes floats), in the handle's INTERNAL node order (see
 *     cm_permutation).  The internal order keeps each cell's nodes
 *     contiguous and in the cell's own range of the input order.
 *   - Every compute call is asynchronous on the given stream, allocates no
 *     memory, and may be captured into a HIP graph.  A handle is not
 *     thread-safe.  Forward calls (cm_forces*) and backward calls
 *     (cm_forces_backward*) use separate scratch memory of the handle, so
 *     one forward and one backward may run concurrently on two streams; two
 *     forward calls (or two backward calls) that overlap race.
 *   - Every call returns CM_OK or a negative status; cm_last_error() gives a
 *     message (thread-local, valid until the next call on that thread).
 *   - Device pointers may not alias each other.
 */
#ifndef CELLMECH_H_
#define CELLMECH_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cm_batch_s* cm_batch;
typedef cm_batch cm_mesh; /* a single-cell handle */

enum {
  CM_OK = 0,
  CM_EINVAL = -1,      /* bad argument (null pointer, size, index, parameter) */
  CM_EDEGENERATE = -2, /* a reference tetrahedron with (near) zero volume */
  CM_EHIP = -3,        /* a HIP runtime call failed */
  CM_ENOMEM = -4,      /* device or host allocation failed */
  CM_ESTATE = -5       /* call out of order (e.g. forces before set_params) */
};

/* Node / tetrahedron ordering used to form tiles. */
/* CM_ORDER_BISECT: tiles by recursive inertial bisection of the reference
 * centroids (compact tiles, fewer shared nodes), Morton order inside a tile. */
enum { CM_ORDER_INPUT = 0, CM_ORDER_RCM = 1, CM_ORDER_MORTON = 2, CM_ORDER_BISECT = 3 };

typedef struct {
  int32_t order;          /* CM_ORDER_*; default CM_ORDER_BISECT             */
  int32_t tile_tets;      /* tetrahedra per tile, a multiple of 64 in        */
                          /* [64, 4096]; 0 = default (768)                    */
  double degenerate_tol;  /* reject |det J| <= tol * h^3 with h the cell's   */
                          /* mean edge length; <= 0 means the default 1e-12  */
} cm_options;

typedef struct {
  int64_t n_cells, n_nodes, n_tets;
  int64_t n_tiles;        /* tiles over all cells                             */
  int64_t n_shared;       /* nodes touched by more than one tile             */
  int64_t n_slots;        /* (tile, shared node) pairs                        */
  int64_t n_chunks;       /* 64-lane chunks over all tiles                    */
  int32_t tile_tets;      /* tetrahedra per tile                              */
  int32_t max_tile_nodes; /* largest number of distinct nodes in one tile     */
  int64_t device_bytes;   /* device memory owned by the handle                */
  double volume;          /* sum of V0 over all cells                         */
  double min_v0;          /* smallest reference volume                        */
  double max_cond;        /* largest 1-norm condition number of J (ref edges) */
  int32_t n_regions;      /* material regions per cell (1 without regions)    */
} cm_info;

/* Message for the last failure on this thread ("" if none). */
const char* cm_last_error(void);

/* Library ABI version (this header: 1). */
int cm_version(void);

/* Fills *opt with the defaults. */
void cm_options_default(cm_options* opt);

/*
 * cm_batch_create: upload the reference meshes of n_cells cells.
 *   node_off, tet_off : host int64[n_cells + 1], CSR offsets (first = 0).
 *   ref_xyz           : host float64[n_nodes * 3], xyz per node (array of
 *                       structures), input node order.
 *   tets              : host int32[n_tets * 4], CELL-LOCAL vertex indices.
 *   opt               : nullable (defaults).
 * Precomputes in FP64 on the host, once (Jacobian paragraph of the paper):
 * B = J^-1 and V0 per tetrahedron, stored as float32; orders and tiles the
 * mesh; copies everything to the device on `stream` and waits for it.
 * Errors: CM_EINVAL (sizes, offsets, an index out of range, repeated vertex
 * in a tetrahedron, a cell without tetrahedra), CM_EDEGENERATE (the message
 * names the cell and tetrahedron), CM_ENOMEM, CM_EHIP.
 * The caller keeps ownership of all host arrays; *out owns its device memory.
 */
int cm_batch_create(int32_t n_cells, const int64_t* node_off,
                    const int64_t* tet_off, const double* ref_xyz,
                    const int32_t* tets, const cm_options* opt,
                    hipStream_t stream, cm_batch* out);

/* Single-cell form of cm_batch_create. */
int cm_mesh_create(int64_t n_nodes, int64_t n_tets, const double* ref_xyz,
                   const int32_t* tets, const cm_options* opt,
                   hipStream_t stream, cm_mesh* out);

/*
 * cm_template_create: n_cells cells that share ONE reference mesh
 * (ref_xyz: host float64[n_nodes * 3], tets: host int32[n_tets * 4]) but have
 * their own deformed positions and parameters.  The precomputed tet data
 * (indices, B, V0) is stored once; the tiles of all cells are interleaved
 * (tile k of every cell, then tile k + 1), so cells running together read the
 * same tet data and HBM sees it about once.  Node arrays hold n_cells blocks
 * of n_nodes nodes (cell c at [c n_nodes, (c + 1) n_nodes) in each SoA
 * component), every block in the same internal order.  Results equal those
 * of cm_batch_create with n_cells copies of the mesh.  The per-cell launch
 * calls return CM_EINVAL on such a handle.  Errors as cm_batch_create.
 * (Several copies of one cell model, as in the paper's suspension runs.)
 */
int cm_template_create(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                       const double* ref_xyz, const int32_t* tets,
                       const cm_options* opt, hipStream_t stream,
                       cm_batch* out);

/*
 * Material regions (the paper notes that the force evaluation is local to a
 * tetrahedron, so parts of a cell such as the nucleus or an actin cortex can
 * carry their own elastic parameters: Sec. "Theory", after eq.
 * elastic-force-vertex-1).  tet_region: host uint8[n_tets], the region of
 * every tetrahedron in input order, each < n_regions; n_regions in [1, 64].
 * Every cell then has n_regions material slots: slot c * n_regions + r holds
 * the (mu, kappa, w) of region r of cell c (cm_set_params) and receives its
 * gradient (cm_forces_backward thetabar, 3 values per slot).  Energies and
 * inverted counts stay per cell.  No tile spans two regions (each region is
 * tiled on its own).  With n_regions = 1 (tet_region may then be NULL) the
 * handle equals the one of cm_batch_create / cm_template_create.  Errors as
 * those, plus CM_EINVAL for a region id >= n_regions.
 */
int cm_batch_create_regions(int32_t n_cells, const int64_t* node_off,
                            const int64_t* tet_off, const double* ref_xyz,
                            const int32_t* tets, const uint8_t* tet_region,
                            int32_t n_regions, const cm_options* opt,
                            hipStream_t stream, cm_batch* out);
int cm_template_create_regions(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                               const double* ref_xyz, const int32_t* tets,
                               const uint8_t* tet_region, int32_t n_regions,
                               const cm_options* opt, hipStream_t stream,
                               cm_batch* out);

/* Frees the handle's device memory and graphs (synchronises the device). */
int cm_destroy(cm_batch h);

int cm_get_info(cm_batch h, cm_info* out);

/* new_to_old: host int64[n_nodes]; entry g is the input-order index of
 * internal node g.  Both orders keep every cell inside its own node range. */
int cm_permutation(cm_batch h, int64_t* new_to_old);

/*
 * cm_set_params: Mooney-Rivlin parameters per material slot (mu, kappa, w),
 * with mu1 = w mu, mu2 = (1 - w) mu (Sec. "Theory").  Arrays hold
 * n_cells * n_regions float64 values each (one per cell without regions); `on_device` = 0 for host arrays (validated, copied;
 * the call waits for the copy), 1 for device arrays (device-to-device copy
 * enqueued on `stream`, graph-safe; values are not validated).
 * Host values must be finite with mu >= 0, kappa >= 0, 0 <= w <= 1, else
 * CM_EINVAL.
 */
int cm_set_params(cm_batch h, const double* mu, const double* kappa,
                  const double* w, int on_device, hipStream_t stream);

/*
 * cm_forces: forces and energies for all cells (eqs. elastic-force-vertex-0
 * and -1, summed over tetrahedra).
 *   y          : device float32[3 * n_nodes] SoA deformed positions.
 *   f          : device float32[3 * n_nodes] SoA forces, overwritten.
 *   energy     : device float64[n_cells] (E = sum V0 U per cell), nullable.
 *   n_inverted : device int32[n_cells], tetrahedra with J <= 0, nullable.
 * Deterministic: the same input gives bitwise the same output.
 * CM_ESTATE before the first cm_set_params.
 */
int cm_forces(cm_batch h, const float* y, float* f, double* energy,
              int32_t* n_inverted, hipStream_t stream);

/*
 * cm_forces_checked: cm_forces plus a per-cell count of tetrahedra whose
 * energy V0 U or force contribution is not finite (NaN or infinite: from
 * non-finite positions, or J = 0 where J^-1/3 is singular).  A node force
 * or a cell energy is non-finite only where such a tetrahedron exists (short
 * of overflow in a sum), so n_nonfinite[c] > 0 flags every cell whose output
 * cannot be used.
 *   n_nonfinite : device int32[n_cells], required.
 * Results (f, energy, n_inverted) are bitwise those of cm_forces; kernels
 * run to completion on any input.  Errors as cm_forces, and CM_EINVAL for a
 * null n_nonfinite.
 */
int cm_forces_checked(cm_batch h, const float* y, float* f, double* energy,
                      int32_t* n_inverted, int32_t* n_nonfinite,
                      hipStream_t stream);

/*
 * cm_forces_noalloc: cm_forces for callers that cannot allocate device
 * memory or must not touch the handle's scratch (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and summation order as cm_forces, so the results are
 * bitwise those of cm_forces; the call allocates and frees nothing.  Its
 * scratch (the shared-node slot partials, 12 B per slot, and per tile an
 * energy and an inverted count, 12 B per tile, each part 256-byte aligned)
 * lives in one static device array of CM_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the library's load until the process ends; its device address
 * is looked up on the first call on each GPU.  Every call on a GPU shares
 * that array and leaves its contents behind (every entry it reads is
 * written first in the same call), so calls that overlap on one GPU -- on
 * two streams, or from two threads, whatever their handles -- race.
 * Errors: as cm_forces, and CM_EINVAL (the message states both sizes) when
 * the handle needs more scratch than the array holds (about 1.3 million
 * slots: a batch of a few hundred cells of the paper's size; larger batches
 * use cm_forces).
 */
#define CM_NOALLOC_SCRATCH_BYTES (16u << 20)
int cm_forces_noalloc(cm_batch h, const float* y, float* f, double* energy,
                      int32_t* n_inverted, hipStream_t stream);

/*
 * cm_forces_backward: reverse-mode cotangents of a loss L(f, E).
 *   fbar     : device float32[3 * n_nodes] = dL/df, nullable (zero).
 *   ebar     : device float64[n_cells] = dL/dE per cell, nullable (zero).
 *   ybar     : device float32[3 * n_nodes] out:
 *              ybar = (df/dy)^T fbar + ebar dE/dy = -H fbar - ebar f with
 *              H the Hessian of E (a Hessian-vector product per cell).
 *   thetabar : device float64[3 * n_cells * n_regions] out, per material
 *              slot (dL/dmu, dL/dkappa, dL/dw); nullable.
 * The paper gives first derivatives only; this is their exact derivative.
 */
int cm_forces_backward(cm_batch h, const float* y, const float* fbar,
                       const double* ebar, float* ybar, double* thetabar,
                       hipStream_t stream);

/*
 * cm_forces_and_backward: cm_forces and cm_forces_backward in one pass over
 * the tetrahedra, for a loss L(f, E) whose cotangents fbar and ebar are
 * known before the forces (a loss linear in f and E, such as
 * L = sum_i v_i . f_i with fixed v).  Forces by eq. elastic-force-vertex-1
 * as for cm_forces; ybar and thetabar as for cm_forces_backward.
 *   y, f, energy, n_inverted : as cm_forces;
 *   fbar, ebar, ybar, thetabar : as cm_forces_backward.
 * Every tetrahedron's deformation gradient, invariants and cofactor matrix
 * are formed once for both results, and each chunk of the mesh is read
 * once; the per-tetrahedron arithmetic and every summation order are those
 * of the two separate calls, so all outputs equal theirs bit for bit.
 * Launch shape: the handle's (cm_set_launch), with waves per workgroup
 * halved until the pass's LDS (48 B per tile node and wave) fits in 64 KiB.
 * Nothing is allocated.  Errors: as cm_forces and cm_forces_backward, and
 * CM_EINVAL if f or ybar equals another of f, ybar, y, fbar (outputs are
 * written while other tiles still read the inputs; buffers that overlap
 * without being equal are not detected and must not be passed).
 */
int cm_forces_and_backward(cm_batch h, const float* y, float* f, double* energy,
                           int32_t* n_inverted, const float* fbar, const double* ebar,
                           float* ybar, double* thetabar, hipStream_t stream);

/*
 * cm_forces_backward_cells: cm_forces_backward restricted to the cells c
 * with cell_flags[c * flag_stride] != 0 (for iterative solvers in which
 * cells finish at different times, e.g. the conjugate gradients of
 * cm_qs_cg_step, whose state column 2 can serve as the flags).
 *   cell_flags  : device float64, read at c * flag_stride for c < n_cells.
 *   flag_stride : >= 1, in elements.
 * For a selected cell, ybar and thetabar are bitwise those of
 * cm_forces_backward; tiles of other cells are not evaluated and their
 * ybar and thetabar entries are left unchanged.  Errors: as
 * cm_forces_backward, and CM_EINVAL for a null cell_flags or a stride < 1.
 */
int cm_forces_backward_cells(cm_batch h, const float* y, const float* fbar,
                             const double* ebar, const double* cell_flags,
                             int64_t flag_stride, float* ybar, double* thetabar,
                             hipStream_t stream);

/*
 * Same results as cm_forces / cm_forces_backward, but one kernel launch per
 * cell (the plain single-cell path).  Used as the comparison baseline of the
 * batched persistent launch.
 */
int cm_forces_percell(cm_batch h, const float* y, float* f, double* energy,
                      int32_t* n_inverted, hipStream_t stream);
int cm_forces_backward_percell(cm_batch h, const float* y, const float* fbar,
                               const double* ebar, float* ybar,
                               double* thetabar, hipStream_t stream);

/*
 * Launch configuration of the batched kernels: waves (tiles) per workgroup
 * (1, 2, 4, 8) and persistent workgroups per compute unit (0 = one workgroup
 * per group of tiles, not persistent).  cm_autotune times one forward +
 * backward evaluation -- the fused pass of cm_forces_and_backward where its
 * LDS fits, else cm_forces then cm_forces_backward -- for every candidate
 * that fits in LDS on `stream`, with the handle's data,
 * the caller's positions `y` (device, SoA, also used as the cotangent) and
 * the parameters already set, and keeps the fastest.  `cache_path`
 * (nullable) is a JSON file keyed by device name, mesh statistics and the
 * timed objective; a hit skips the measurement, a miss appends the result.
 * Tuning allocates and
 * frees scratch outputs and synchronises the stream: it is not graph-safe.
 */
/*
 * cm_batch_create_tuned: cm_batch_create with the tile size chosen by
 * measurement.  For every candidate tile size (tile_candidates, host
 * int32[n_candidates], multiples of 64 in [64, 4096]; NULL = {512, 640, 768,
 * 896, 1024}) the meshes are prepared and uploaded, and one forward +
 * backward evaluation is timed as in cm_autotune for every launch
 * configuration, with the
 * reference positions as input and unit parameters (the work per
 * tetrahedron does not depend on them); the fastest tile size and launch
 * are kept, the other handles freed as soon as they lose.  candidate_ms
 * (host float64[n_candidates], nullable) receives each candidate's best
 * time (infinity where skipped).  cache_path (nullable): a JSON file of the
 * cm_autotune format keyed by device, cell / node / tetrahedron counts,
 * ordering and candidate list; a hit prepares only the cached tile size.
 * opt->tile_tets is ignored.  cm_set_params must still be called on the
 * result.  Allocates and synchronises; one handle of every candidate is
 * alive at a time beside the best so far.  Errors as cm_batch_create, and
 * CM_EINVAL for a bad candidate list.
 */
int cm_batch_create_tuned(int32_t n_cells, const int64_t* node_off,
                          const int64_t* tet_off, const double* ref_xyz,
                          const int32_t* tets, const cm_options* opt,
                          const int32_t* tile_candidates, int32_t n_candidates,
                          const char* cache_path, double* candidate_ms,
                          hipStream_t stream, cm_batch* out);

int cm_set_launch(cm_batch h, int32_t waves_per_block, int32_t blocks_per_cu);
int cm_get_launch(cm_batch h, int32_t* waves_per_block, int32_t* blocks_per_cu);
int cm_autotune(cm_batch h, const float* y, const char* cache_path,
                hipStream_t stream);

/*
 * HIP graph of one batched evaluation with fixed buffers.
 *   mode 0: forward (cm_forces);
 *   mode 1: forward then backward (cm_forces, cm_forces_backward);
 *   mode 2: the per-cell launches of mode 0 (single-cell baseline);
 *   mode 3: the per-cell launches of mode 1;
 *   mode 4, 5: as 1, 3 but with the backward pass as a parallel branch of
 *   the graph (it reads y, fbar and ebar only and has its own scratch), so
 *   the two passes may overlap on the device;
 *   mode 6: forward and backward in one pass (cm_forces_and_backward).
 * Pointers are captured as given and must stay valid while the graph is
 * used.  Re-capturing replaces the previous graph.  cm_graph_launch replays
 * it on `stream` (CM_ESTATE if nothing was captured).
 */
int cm_graph_capture(cm_batch h, int mode, const float* y, float* f,
                     double* energy, int32_t* n_inverted, const float* fbar,
                     const double* ebar, float* ybar, double* thetabar,
                     hipStream_t stream);
int cm_graph_launch(cm_batch h, hipStream_t stream);

/*
 * Plate compression (time-stepped relaxation).  The paper compresses cells
 * between a resting and a moving plate with a repulsive force that keeps
 * vertices out of the plates (Sec. "Simulation setup"); the force law and
 * the time integration are in its unavailable supporting information.
 * This library implements the reading (overdamped explicit steps, quadratic
 * penalty):
 *   p_z = -k max(0, y_z - top_c)^2 + k max(0, bottom_c - y_z)^2,
 *   y_next = y + m (f + p),   force[c] = k sum_{nodes of c} max(0, y_z - top_c)^2,
 * with f the elastic forces of cm_forces for the same y, k = k_plate and
 * m = mobility (time step over drag).
 *   plate   : device float64[2 * n_cells], (top_c, bottom_c) per cell.
 *   y, f    : device float32[3 * n_nodes] SoA; y_next likewise (no aliasing).
 *   force   : device float64[n_cells] out, nullable.
 * cm_plate_step_adjoint gives the reverse-mode step for a loss that adds
 * scale * (F_meas[c] - F_target[c])^2 per cell at this step (F_target
 * nullable = no loss term, F_meas = the force of cm_plate_step at y):
 *   lam = lam_next + m ((df/dy)^T lam_next + dp/dy lam_next)
 *         + 2 scale (F_meas - F_target) dF/dy,
 * where ybar_el = (df/dy)^T lam_next is cm_forces_backward(y, fbar =
 * lam_next); and, if given, thetabar_acc[q] += m thetabar_el[q] for the
 * 3 n_regions entries q of every cell
 * (thetabar_el from the same cm_forces_backward call).  lam must not alias
 * any input.  Errors: CM_EINVAL for null/aliased pointers or negative or
 * non-finite k_plate / mobility.
 */
int cm_plate_step(cm_batch h, const float* y, const float* f,
                  const double* plate, double k_plate, double mobility,
                  float* y_next, double* force, hipStream_t stream);
int cm_plate_step_adjoint(cm_batch h, const float* y, const float* lam_next,
                          const float* ybar_el, const double* plate,
                          double k_plate, double mobility,
                          const double* F_meas, const double* F_target,
                          double scale, const double* thetabar_el,
                          double* thetabar_acc, float* lam,
                          hipStream_t stream);

/*
 * The same plate-compression steps with the elastic forces computed inside
 * the step (one force pass whose epilogue applies the step, instead of
 * cm_forces followed by cm_plate_step, and one adjoint pass instead of
 * cm_forces_backward followed by cm_plate_step_adjoint): the intermediate f,
 * ybar_el and thetabar_el are never stored.  Same reading and arguments as
 * above.  The per-node arithmetic is that of the two-call route: y_next,
 * lam, thetabar_acc, energy and inverted counts are bitwise equal to it.
 * The top-plate force sums the same float64 node terms in another fixed
 * order (each tile's share, then the nodes of no tetrahedron), so it agrees
 * to rounding and is bitwise repeatable.
 *   cm_plate_forces_step: y_next, force (nullable) and, if given, the
 *     per-cell energy and inverted count of cm_forces at y.
 *   cm_plate_backward_step: lam from lam_next (the cotangent of the forces
 *     pass is lam_next, with no energy cotangent); if thetabar_acc is given,
 *     thetabar_acc[q] += m thetabar_el[q] for the 3 n_regions entries of
 *     every cell.
 * y_next and lam must not alias the inputs.  Errors: CM_EINVAL for null or
 * aliased pointers, negative or non-finite k_plate / mobility, non-finite
 * scale, F_target without F_meas, a launch configuration beyond the LDS;
 * CM_ESTATE before cm_set_params.
 */
int cm_plate_forces_step(cm_batch h, const float* y, const double* plate,
                         double k_plate, double mobility, float* y_next,
                         double* force, double* energy, int32_t* n_inverted,
                         hipStream_t stream);
int cm_plate_backward_step(cm_batch h, const float* y, const float* lam_next,
                           const double* plate, double k_plate, double mobility,
                           const double* F_meas, const double* F_target,
                           double scale, double* thetabar_acc, float* lam,
                           hipStream_t stream);

/*
 * Quasi-static plate compression (the compression setup of Sec. "Simulation
 * setup" solved for equilibrium instead of stepped in time).  At plate
 * positions plate[2c] = top, plate[2c + 1] = bottom the state of cell c
 * minimises Pi(y) = E(y) + sum_nodes (k/3) [max(0, y_z - top)^3 +
 * max(0, bottom - y_z)^3] (the potential of the penalty of cm_plate_step), so
 * that f + p = 0.  A Newton step solves Hess(Pi) dx = f + p per cell by
 * conjugate gradients whose Hessian-vector products are cm_forces_backward
 * calls (ybar = (df/dy)^T v = -Hess(E) v) plus the diagonal penalty
 * Hessian; the caller drives the loop:
 *   cm_forces(y -> f, E); cm_qs_residual;  repeat: cm_forces_backward(y,
 *   fbar = p -> ybar); cm_qs_cg_step;  then either cm_qs_update (bounded
 *   step) or a line search on Pi: cm_qs_ls_start, then repeat cm_forces(
 *   y_trial -> E_trial); cm_qs_ls_accept while some cell is pending.
 * Arrays (device, SoA float32[3 n_nodes]): r (residual), p (search
 * direction), x (Newton step), Ap (scratch), r_newton (copy of r_N,
 * nullable), y_trial; state: float64[16 n_cells] = CG r . z (|r|^2 without
 * preconditioner), CG |r_0|^2, CG
 * active, |r_N|^2, accepted step scale, |penalty|^2, largest node move of
 * the last step, float32 floor rho, Pi(y), line-search scale, slope
 * r_N . x, not in equilibrium (1/0), line search pending (1/0), max |x|,
 * CG forcing term eta, |r_N|^2 of the last residual.
 *   cm_qs_residual: r = p = r_N, x = 0, with r_N = f + penalty minus its
 *     components along the exact symmetries of the plates (translations in
 *     x and y, rotation about z through the centroid); active iff |r_N|_2 >
 *     max(abs_tol, rel_tol |penalty|_2, floor_factor rho) and the last step
 *     moved some node by more than step_tol (restart != 0: no last step, at
 *     a new plate position; under the sphere the residual also loses its
 *     lateral mean, the held centroid's force); force (nullable)
 *     float64[2 n_cells] = top (the sphere's, under the sphere) and
 *     bottom plate forces k sum max(0, .)^2; energy (nullable) E(y) per cell
 *     from cm_forces, giving Pi(y) in the state.  eta_max in [0, 1): with
 *     eta_max > 0 the Newton step is inexact (Eisenstat and Walker's second
 *     forcing term): eta = 0.9 (|r_N| / |r_N,prev|)^2, at least 0.9
 *     eta_prev^2 when that exceeds 0.1, at least half of tolerance / |r_N|,
 *     at most eta_max (eta_max at a new plate position); eta_max = 0 sets
 *     eta = 0.
 *   cm_qs_ls_start: for cells not in equilibrium, x is first projected in
 *     place onto the complement of the symmetry modes (its mean x and y
 *     components and its rotation about z through the centroid of y are
 *     removed: Hess(Pi) annihilates them, so the CG leaves whatever its
 *     preconditioned directions put there); then s = min(1, cap /
 *     max_i |x_i|), slope r_N . x; y_trial = y + s x for cells not in
 *     equilibrium whose step descends, y otherwise.
 *   cm_qs_ls_accept (energy_trial = E(y_trial) from cm_forces): a pending
 *     cell accepts y_trial (copied into y) if Pi(y_trial) <= Pi(y) - armijo
 *     s (r_N . x), else halves s and forms the next trial; it gives up (no
 *     move, last step 0) once s max|x| < min_move.  With the inverted counts
 *     (device int32[n_cells] each, both or neither: n_inverted_trial from
 *     cm_forces at y_trial, n_inverted those at y, updated on acceptance) a
 *     trial that inverts more tetrahedra than y has is rejected too (the
 *     energy density grows without bound as J -> 0 from above; a finite step
 *     could jump over that barrier to an inverted state of finite energy).
 *   cm_qs_noise / cm_qs_floor: the float32 floor rho of the residual: e =
 *     +-|y| 2^-24 per coordinate (half a unit in the last place, signs from
 *     a fixed hash of the index), then after ybar = cm_forces_backward(y,
 *     fbar = e), rho = |Hess(Pi) e|_2 per cell, stored in the state.
 *   cm_qs_stiffness: k_el (device float32[6 n_nodes] SoA: xx, yy, zz, xy,
 *     xz, yz) = per node the sum over its tetrahedra of the diagonal 3x3
 *     block of the small-strain stiffness, V0 (mu |b|^2 I + (kappa + mu/3)
 *     b b^T) with b the node's row of the tetrahedron's gradient operator
 *     (B's rows, minus their sum for vertex 4) and (mu, kappa) of its
 *     material slot: the small-strain limit of the energy (shear modulus
 *     mu, bulk modulus kappa), used as a block-Jacobi preconditioner.
 *     Uses the forward scratch (do not overlap with cm_forces); CM_ESTATE
 *     before cm_set_params.
 *   cm_qs_residual with k_el and minv (device float32[6 n_nodes], both or
 *     neither): minv = the inverse of k_el plus the penalty Hessian per
 *     node (identity where that block is not positive definite), and the
 *     CG starts from p = minv r (preconditioned CG).
 *   cm_qs_cg_step: one CG iteration for every active cell, preconditioned
 *     by minv (nullable: plain CG; pass the array cm_qs_residual filled); a
 *     cell stops at |r| <= max(rel_tol, eta) |r_0| or at non-positive
 *     curvature.  Under the sphere the contact Hessian is a 3x3 block per
 *     node and Hess(Pi) p and the preconditioned direction are projected
 *     like the residual (see cm_qs_set_indenter).
 *   cm_qs_update: y += s x per cell, s = min(1, cap / m) with m the
 *     largest |component| of x over the cell's nodes; for a cell with m > 0,
 *     state[4] = s and state[6] = m s (its largest coordinate move).
 *   cm_qs_predict: z -> b' + (z - b) s, s = (t' - b') / (t - b), for a new
 *     plate pair (t', b'), and x, y stretched by 1/sqrt(s) about the cell's
 *     centroid (a volume-preserving affine prediction).
 * Errors: CM_EINVAL for null pointers, negative or non-finite k_plate or
 * tolerances, cap <= 0, eta_max outside [0, 1).
 */
/*
 * cm_qs_set_indenter: the top contact of the quasi-static entry points of
 * this handle (Sec. "Simulation setup": two plates, or a sphere indenting
 * the cell as in the colloidal-probe comparison of Sec. "Validation with
 * AFM experiments").  radius = 0 (the default): the flat top plate at
 * plate[2c].  radius > 0: a sphere of that radius whose lowest point is at
 * plate[2c] and whose vertical axis passes through (axis_xy[2c],
 * axis_xy[2c + 1]) (device float64[2 n_cells], copied on `stream`).  The
 * sphere repels nodes with the plates' penalty law in the penetration depth
 * g = max(0, radius - |y - c|): potential (k/3) g^3, force k g^2 n along the
 * unit vector n from the centre, the force on the sphere k sum g^2 (c_z -
 * y_z) / |y - c| upward (reported as the top force).  Frictionless contacts
 * leave sliding off the sphere's axis unstable, so under the sphere each
 * cell's centroid is held laterally: the residual, the CG iterates (the
 * Hessian-vector products and preconditioned directions), the adjoint's
 * right-hand side and the Newton step lose their lateral translation and
 * their rotation about the vertical axis through the centroid.  cm_qs_update
 * and cm_qs_predict are the same for both contacts.  Errors: CM_EINVAL for a
 * negative or non-finite radius, or a sphere without axis_xy.
 */
int cm_qs_set_indenter(cm_batch h, double radius, const double* axis_xy,
                       hipStream_t stream);

int cm_qs_residual(cm_batch h, const float* y, const float* f, const double* energy,
                   const double* plate, double k_plate, double abs_tol,
                   double rel_tol, double step_tol, double floor_factor,
                   double eta_max, int32_t restart, float* r, float* p, float* x,
                   float* r_newton, double* state, double* force, const float* k_el,
                   float* minv, hipStream_t stream);
int cm_qs_stiffness(cm_batch h, float* k_el, hipStream_t stream);
/*
 * cm_qs_adjoint_rhs: start of the adjoint solve for the derivative of the
 * top-plate force at an equilibrium (f + p = 0) with respect to the
 * material parameters: dF_top/dtheta = lam^T df/dtheta with
 * Hess(Pi) lam = g, g = dF_top/dy (2 k max(0, y_z - top) on the z entries).
 * Sets r = weight[c] g (weight: device float64[n_cells], nullable = 1),
 * p = minv r (minv nullable: p = r; pass the blocks of the last
 * cm_qs_residual at this y), x = 0, and the CG columns of the state (r . z,
 * |r|^2, active iff |r| > 0, forcing term 0).  The caller then runs the CG
 * loop of a Newton step (cm_forces_backward_cells + cm_qs_cg_step, which
 * stop at cg_tol) and gets lam in x; cm_forces_backward(y, fbar = lam) then
 * gives thetabar = weight dF_top/d(mu, kappa, w) per material slot.  Under
 * the plates g has z entries only, so it is orthogonal to the symmetry modes
 * (translations in x and y, rotation about z) and the singular system is
 * consistent.  Under the sphere (cm_qs_set_indenter) F_top = k sum g_s^2 m
 * with g_s the penetration and m = (c_z - y_z) / |y - c|, so g = -k (2 g_s m n
 * + (g_s^2 / |y - c|)(e_z + m n)) per node; r and p are projected onto the
 * complement of the lateral translations and the vertical rotation (the
 * held centroid), as the CG keeps its iterates there; pass the blocks and
 * positions of the last cm_qs_residual (its centroids are used).  Errors:
 * CM_EINVAL for null pointers or a negative or non-finite k_plate.
 */
int cm_qs_adjoint_rhs(cm_batch h, const float* y, const double* plate, double k_plate,
                      const double* weight, float* r, float* p, float* x, double* state,
                      const float* minv, hipStream_t stream);
int cm_qs_ls_start(cm_batch h, float* x, const float* r_newton, double cap,
                   const float* y, float* y_trial, double* state,
                   hipStream_t stream);
int cm_qs_ls_accept(cm_batch h, const float* x, const double* plate, double k_plate,
                    const double* energy_trial, double armijo, double min_move,
                    float* y, float* y_trial, double* state,
                    const int32_t* n_inverted_trial, int32_t* n_inverted,
                    hipStream_t stream);
int cm_qs_noise(cm_batch h, const float* y, float* e, hipStream_t stream);
int cm_qs_floor(cm_batch h, const float* y, const double* plate, double k_plate,
                const float* e, const float* ybar, double* state, hipStream_t stream);
int cm_qs_cg_step(cm_batch h, const float* y, const double* plate, double k_plate,
                  double rel_tol, const float* ybar, float* x, float* r, float* p,
                  float* Ap, double* state, const float* minv, hipStream_t stream);
/*
 * cm_qs_cg_iteration: one CG iteration with its Hessian-vector product in a
 * single call, the same as cm_forces_backward_cells(y, fbar = p, cells =
 * state column 2) followed by cm_qs_cg_step, with bitwise the same x, r, p
 * and state: the backward tile pass stores the owned nodes' (df/dy)^T p in
 * ybar (device float32[3 n_nodes], caller-owned scratch) and leaves the
 * shared nodes' partials in the handle's backward scratch, whose sums the CG
 * kernel forms itself in the finalize's order (one launch and one pass over
 * the shared nodes fewer per iteration).  Uses the backward scratch (do not
 * overlap with cm_forces_backward*).  Errors: as cm_qs_cg_step, CM_ESTATE
 * before cm_set_params, CM_EINVAL for a launch beyond the LDS.
 */
int cm_qs_cg_iteration(cm_batch h, const float* y, const double* plate, double k_plate,
                       double rel_tol, float* ybar, float* x, float* r, float* p,
                       float* Ap, double* state, const float* minv, hipStream_t stream);
int cm_qs_update(cm_batch h, const float* x, double cap, float* y, double* state,
                 hipStream_t stream);
int cm_qs_predict(cm_batch h, const double* plate_old, const double* plate_new,
                  float* y, hipStream_t stream);

/*
 * cm_shape: deformation diagnostics of every cell at positions y.
 *   Taylor deformation parameter D = (a3 - a1) / (a3 + a1) (Sec. "Taylor
 *   deformation parameter", eq. taylor-deformation-parameter-definition)
 *   from the discretised inertia tensor I = sum_l V_l (|r_l|^2 1 - r_l r_l^T)
 *   (eq. inertia-tensor-discretized; V_l the current volume of tetrahedron
 *   l with its reference orientation, r_l its centroid, taken about the
 *   cell's centre of mass) and the semi-axes of eq.
 *   inertia-tensor-ellipsoid-semiaxes read as squared semi-axes
 *   (a_i = sqrt(5 / (2 M) (...)), M the current volume, 0 if negative);
 *   cell strain (d_max - d_ref) / d_ref (eq. cell-strain) with d_max the
 *   largest distance between two nodes of the cell.
 *   y     : device float32[3 * n_nodes] SoA positions.
 *   d_ref : device float64[n_cells] reference diameters (2 R for the paper's
 *           spherical cell), nullable: strain = NaN.
 *   out   : device float64[n_cells * 10], per cell: volume, centre of mass
 *           (x, y, z), a1 <= a2 <= a3, D, d_max, strain.
 * All sums in float64 in a fixed order (deterministic).  Errors: CM_EINVAL
 * for null y / out or tiles whose nodes exceed 64 KiB of LDS (16 B each).
 */
int cm_shape(cm_batch h, const float* y, const double* d_ref, double* out,
             hipStream_t stream);

/*
 * cm_profile_kernels: average device time of each kernel of one batched
 * forward + backward evaluation, measured with HIP events recorded on
 * `stream` around `reps` back-to-back launches of each kernel:
 *   ms[0] forward tile kernel,  ms[1] forward finalize kernel,
 *   ms[2] backward tile kernel, ms[3] backward finalize kernel,
 *   ms[4] tile kernel and ms[5] finalize kernel of cm_forces_and_backward
 *         (NaN where that pass does not apply: aliased buffers or too
 *         little LDS).
 * Buffers as in cm_forces / cm_forces_backward (fbar, ebar nullable);
 * ms holds 6 entries.
 * Synchronises the stream; not graph-safe.
 */
int cm_profile_kernels(cm_batch h, const float* y, float* f, double* energy,
                       const float* fbar, const double* ebar, float* ybar,
                       double* thetabar, int32_t reps, double* ms,
                       hipStream_t stream);

/*
 * cm_stream_copy: dst[i] = src[i] for i < n (device float arrays, n >= 0; no
 * overlap), one dword per lane per load instruction like the tile kernels'
 * chunk stream, asynchronous on `stream`.  A kernel of known traffic (4 n
 * bytes read, 4 n written) against which hardware byte counters are scaled.
 * Errors: CM_EINVAL for n < 0 or null pointers with n > 0.
 */
int cm_stream_copy(const float* src, float* dst, int64_t n, hipStream_t stream);

/*
 * Host-only view of the prepared layout (no device work), for validation and
 * debugging of the preparation step.  cm_layout_create runs exactly the
 * preparation of cm_batch_create (same arguments, same errors).
 * cm_layout_sizes fills sizes[8] = {n_tiles, n_chunks, n_slots, n_shared,
 * n_nodes, n_cells, max_tile_nodes, tile_tets}.  cm_layout_export copies the
 * tables into caller-owned host arrays (each nullable):
 *   tiles        int32[n_tiles * 8]   (chunk_begin, n_tets, own_begin, n_own,
 *                                      shr_begin, n_shr, cell, n_chunks)
 *   chunks       uint8[n_chunks * 3072] (64 tetrahedra each, three rows of
 *                                      64 16-byte records: uint32 a[64][4] =
 *                                      (v0 | v1 << 16, v2 | v3 << 16 local
 *                                      indices in vertex-slot order, bits of
 *                                      float V0, bits of float B[0]), float
 *                                      b[64][4] = B[1..4], float c[64][4] =
 *                                      B[5..8] (B row-major); 0xffffffff in
 *                                      a[lane][0] for an empty lane)
 *   slot_node    int32[n_slots]       shared_node   int32[n_shared]
 *   shared_slot_ptr int32[n_shared+1] shared_slots  int32[n_slots]
 *   cell_tile_off   int32[n_cells+1]  cell_shared_off int32[n_cells+1]
 *   new_to_old      int64[n_nodes]
 * cm_layout_create_template runs the preparation of cm_template_create (same
 * arguments minus the stream, same errors); its layout leaves cell_tile_off
 * untouched (the tiles of cell c are c + k n_cells, k = 0, 1, ...).
 */
typedef struct cm_layout_s* cm_layout;
int cm_layout_create(int32_t n_cells, const int64_t* node_off,
                     const int64_t* tet_off, const double* ref_xyz,
                     const int32_t* tets, const cm_options* opt,
                     cm_layout* out);
int cm_layout_create_template(int32_t n_cells, int64_t n_nodes, int64_t n_tets,
                              const double* ref_xyz, const int32_t* tets,
                              const cm_options* opt, cm_layout* out);
/* The preparation of cm_batch_create_regions; cm_layout_export_regions
 * copies tile_mat int32[n_tiles] (material slot of every tile) and the tiles
 * of every slot, mat_tile_first / mat_tile_count int32[n_cells * n_regions]
 * (tiles first + k, k < count). */
int cm_layout_create_regions(int32_t n_cells, const int64_t* node_off,
                             const int64_t* tet_off, const double* ref_xyz,
                             const int32_t* tets, const uint8_t* tet_region,
                             int32_t n_regions, const cm_options* opt,
                             cm_layout* out);
int cm_layout_export_regions(cm_layout l, int32_t* tile_mat,
                             int32_t* mat_tile_first, int32_t* mat_tile_count);
int cm_layout_sizes(cm_layout l, int64_t* sizes);
int cm_layout_export(cm_layout l, int32_t* tiles, void* chunks,
                     int32_t* slot_node, int32_t* shared_node,
                     int32_t* shared_slot_ptr, int32_t* shared_slots,
                     int32_t* cell_tile_off, int32_t* cell_shared_off,
                     int64_t* new_to_old);
int cm_layout_destroy(cm_layout l);

#ifdef __cplusplus
}
#endif

#endif /* CELLMECH_H_ */
