/*
 * isoadv.h — C interface of the MI355X (gfx950) isoAdvector advection step.
 *
 * The operation (Vukcevic, Roenby, Gatin & Jasak, "A sharp free surface finite
 * volume method applied to gravity wave flows", Section 3.2, problem statement):
 * from the cell volume fractions alpha_P(t), the cell velocities U_P and the
 * volumetric face fluxes phi_f, predict alpha_P(t + dt) by the flux-form update
 *     alpha_P(t+dt) = alpha_P(t) - (1/V_P) sum_f dV_f,
 * where dV_f = phi_f * (time integral over the step of the submerged area
 * fraction of face f) is obtained by sweeping the upwind interface cell's
 * isoface across the face (Eqs. dV, alphaf, tv, x_41, aplus1, aplus2,
 * intaplus), and dV_f = alpha_upwind * phi_f * dt when the upwind cell is not an
 * interface cell (the special cases after Eq. dVdef).  The isoface of a cell is
 * the isosurface of the vertex-interpolated volume fraction (inverse
 * centre-to-vertex distance weights) whose sub-cell volume equals alpha_P V_P.
 * A bounding step (volume-preserving redistribution, then optional chopping to
 * [0,1]) ends the step (last paragraph of Section 3.2).
 *
 * Conventions
 *  - Meshes are face based (points; faces as point lists; owner of every face;
 *    neighbour of every interior face), interior faces first, boundary faces
 *    grouped into patches.  The points of a face run counter-clockwise seen
 *    from outside its owner, so phi_f > 0 is flow from owner to neighbour (or
 *    out of the domain).  Cells (Section 3: arbitrary polyhedra), mixed
 *    freely: hexahedra (6 quadrilateral faces, 8 points); cells of 4 to 6
 *    faces of 3 or 4 points over at most 8 points (tetrahedra, square
 *    pyramids, triangular prisms); and general polyhedra of 4 to 16 faces of 3
 *    to 16 points over at most 32 points (e.g. hexahedra merged across split
 *    faces).  Larger cells give ISO_EUNSUPPORTED.  Every entry point takes
 *    every cell type.
 *  - Patch kinds: WALL and EMPTY faces carry no flux (their phi is ignored);
 *    INOUT faces carry flux, inflow carrying the patch's alpha_in; CYCLIC
 *    patches come in pairs (face n of a patch matches face n of its partner,
 *    x_partner = x_this + translation).  For a cyclic pair the flux is read from
 *    the face of the patch with the lower index (positive: out of that face's
 *    owner); the partner face's phi entry is ignored.
 *  - Arrays passed to iso_mesh_create are HOST arrays, copied; the caller keeps
 *    ownership.  Arrays passed to the step functions are DEVICE arrays owned by
 *    the caller (e.g. torch tensors), read/written on the plan's HIP stream.
 *    Step calls are asynchronous unless a stats pointer is given.
 *  - Every function returns a status; nothing aborts or throws across the
 *    interface.  iso_last_error() gives a message for the last failure on the
 *    calling thread.  A device fault surfaces as ISO_EDEVICE.
 *  - FP64 throughout.  Indices are int32 (meshes up to 2^31-1 faces).
 */
#ifndef ISOADV_H
#define ISOADV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ISO_OK = 0,
    ISO_EINVAL = 1,        /* bad argument (null, size, aliasing, non-finite dt, ...) */
    ISO_ENOMEM = 2,        /* device or host allocation failed */
    ISO_EDEVICE = 3,       /* HIP runtime error or device fault */
    ISO_ENOSPACE = 4,      /* interface cells exceed the plan's capacity */
    ISO_ECOURANT = 5,      /* input check: a cell Courant number exceeds max_courant */
    ISO_EMESH = 6,         /* inconsistent mesh (indices, orientation, cyclic matching, volume) */
    ISO_EUNSUPPORTED = 7   /* valid input the kernels do not take (e.g. a cell of more than 32 points) */
} iso_status;

enum { ISO_PATCH_WALL = 0, ISO_PATCH_EMPTY = 1, ISO_PATCH_INOUT = 2, ISO_PATCH_CYCLIC = 3 };

typedef struct iso_mesh iso_mesh;
typedef struct iso_plan iso_plan;

typedef struct {
    double eps_surf;        /* interface cell iff eps < alpha < 1-eps (default 1e-8) */
    double flat_tol;        /* max-min vertex value at or below which an interface cell is
                               treated as bulk (default 1e-12) */
    double bound_tol;       /* excursions of alpha beyond [−tol, 1+tol] are redistributed;
                               smaller ones are chopped when clip is on (default 1e-12) */
    double max_courant;     /* limit for check_inputs (default 1.0) */
    int32_t root_max_iter;  /* isovalue iterations (default 100) */
    int32_t n_bound_iter;   /* Jacobi redistribution sweeps (default 3) */
    int32_t clip;           /* chop alpha to [0,1] after redistribution (default 1) */
    int32_t check_inputs;   /* validate inputs on the host before each step (syncs; default 0) */
    int32_t block_cells;    /* threads per block of the per-cell kernels, up to 1024 (0 = 256) */
    int32_t surface_blocks; /* work-groups of the interface-cell kernel, which loops over the list
                               (0 = up to 2048, from the list capacity); at most 65535 */
    int32_t max_surface;    /* capacity of the interface-cell list (0 = n_cells) */
    int32_t surface_waves;  /* register budget of the interface-cell kernel in waves per SIMD:
                               1, 2, 3 or 4 (0 = 2) */
    int32_t bound_blocks;   /* work-groups of the bounding sweeps (0 = 512); at most 65535.
                               Results are bitwise the same for every choice of the launch shapes
                               block_cells, surface_blocks, surface_waves and bound_blocks. */
    int32_t us_mode;        /* isoface velocity U_S (Section 3.2 interpolates the cell velocity to
                               the isoface centre x_S and names no scheme): 0 = U_P, the cell value
                               (default); 1 = cell-point interpolation: point velocities with the
                               inverse-distance weights of the vertex values, the cell split into
                               tetrahedra (cell centre, vertex mean of a face, two consecutive face
                               points) carrying U_P, the face's mean point velocity and the point
                               velocities, and the linear interpolant at x_S in the tetrahedron
                               with the largest smallest barycentric coordinate.  The adjoint
                               takes us_mode 0 only (ISO_EUNSUPPORTED). */
    double root_tol;        /* isovalue tolerance (Section 3.2 leaves it to the user): the search
                               stops once |V_sub/V_P - alpha_P| <= root_tol; 0 (default) converges
                               to round-off.  In [0, 1). */
    int32_t full_slots;     /* 1: the update reads every flux slot from the mesh's full-width
                               tables; 0 (default): from its 32-bit slot words where the mesh has
                               them (iso_mesh_info).  The same bits either way. */
} iso_options;

typedef struct {
    int64_t n_surface;       /* interface cells this step */
    int64_t n_flat;          /* interface cells treated as bulk (flat vertex data) */
    int64_t n_nonconverged;  /* isovalue searches that hit root_max_iter */
    int64_t n_bound_active;  /* cells needing redistribution in the first sweep */
    int32_t max_root_iter;
    int32_t reserved;
    double vol_before, vol_after;  /* sum of alpha V before and after the step */
    double vol_boundary_flux;      /* volume that left through boundary faces (inflow negative), with the
                                      redistribution's corrections of boundary faces */
    double vol_clipped;            /* volume the chops added (negative: removed), so that
                                      vol_after = vol_before - vol_boundary_flux + vol_clipped */
    double alpha_min, alpha_max;
} iso_step_stats;

/* Optional per-step intermediates (DEVICE pointers, each may be NULL), for testing. */
typedef struct {
    double *vert_alpha;   /* [8*n_cells] vertex values of interface cells, canonical vertex order */
    int32_t *kind;        /* [n_cells] 0 bulk, 1 reconstructed interface cell, 2 flat interface cell */
    double *iso;          /* [n_cells] isovalue of reconstructed cells */
    double *rec;          /* [7*n_cells] isoface centre x_S (3), unit normal n_S (3), U_S.n_S */
    double *dV;           /* [n_faces] dV per flux face (indexed by the face that carries its phi) */
    double *alpha_raw;    /* [n_cells] alpha after the update, before bounding */
    int32_t *iters;       /* [n_cells] isovalue iterations */
} iso_trace;

void iso_options_default(iso_options *opt);
const char *iso_status_string(iso_status s);
const char *iso_last_error(void);

/* Mesh setup (once, host arrays, copied).  Section 3: collocated polyhedral mesh with
 * owner/neighbour connectivity.  Builds the device geometry of the step. */
iso_status iso_mesh_create(int32_t n_points, const double *px, const double *py, const double *pz,
                           int32_t n_faces, const int32_t *face_ptr /* [n_faces+1] */,
                           const int32_t *face_pts, const int32_t *owner /* [n_faces] */,
                           int32_t n_internal, const int32_t *neighbour /* [n_internal] */, int32_t n_cells,
                           int32_t n_patches, const int32_t *patch_start, const int32_t *patch_size,
                           const int32_t *patch_kind, const int32_t *patch_partner /* -1 if not cyclic */,
                           const double *patch_translation /* [3*n_patches] */,
                           const double *patch_alpha_in /* [n_patches] */, iso_mesh **out);
void iso_mesh_destroy(iso_mesh *mesh);
/* info[0..7] = n_cells, n_points, n_faces, n_flux_faces, n_point_classes, slots per cell,
 *              device bytes held, and the flux slots that the update reads from the full-width
 *              tables beside its 32-bit slot words (-1: the mesh has no such words, because more
 *              than a tenth of its flux slots would not fit them; they fit where the internal
 *              faces are numbered by owner, each owner below its neighbour, and neighbours lie
 *              within 32768 cells) */
iso_status iso_mesh_info(const iso_mesh *mesh, int64_t *info);
/* host out[8*n_cells]: user point id of each canonical vertex of each cell (hexahedra: the
 * canonical order; other cells: their distinct points in order of first appearance over their
 * faces, then the first point repeated) */
iso_status iso_mesh_cell_points(const iso_mesh *mesh, int32_t *out);
/* host out[n_cells]: cell volumes; xc (nullable) [3*n_cells]: cell centres */
iso_status iso_mesh_geometry(const iso_mesh *mesh, double *vol, double *xc);

/* Plan: options, workspace (sized for max_surface interface cells) and the HIP stream
 * (hipStream_t passed as void*, NULL = default stream).  The mesh must outlive the plan. */
iso_status iso_plan_create(const iso_mesh *mesh, const iso_options *opt, void *hip_stream, iso_plan **out);
iso_status iso_plan_set_stream(iso_plan *plan, void *hip_stream);
void iso_plan_destroy(iso_plan *plan);

/* One advection step (Section 3.2).  alpha [n_cells], phi [n_faces], U structure-of-arrays
 * [3*n_cells] (all Ux, then Uy, then Uz), alpha_new [n_cells]: device arrays; alpha_new must
 * not overlap alpha, phi or U.  stats (host, nullable): filled after a device sync. */
iso_status iso_advect_step(iso_plan *plan, const double *alpha, const double *phi, const double *U, double dt,
                           double *alpha_new, iso_step_stats *stats);

/* n_steps advection steps in place (Section 3.2, repeated), for callers that advance one mesh
 * many steps: alpha [n_cells] (device) holds the state before and after.  Step k reads
 * phi + k*phi_stride [n_faces] and U + k*U_stride [3*n_cells] (strides in elements: 0 = the same
 * fields every step, else at least one step's fields).  Bit for bit n_steps calls of
 * iso_advect_step.  A run of up to 256 steps is captured once as a HIP graph and replayed while
 * alpha, the fields, the strides, dt and n_steps stay the same (one call, and a graph a caller's
 * own capture can hold; on the 3D workload as fast as separate steps, not faster); it runs on a
 * stream of the plan's own, ordered after the work before it on the plan's stream and before the
 * work after it.  The first run allocates a
 * second state buffer of n_cells doubles, held until the plan is destroyed.  Not with check_inputs
 * (ISO_EINVAL) or a limited max_surface (ISO_EUNSUPPORTED); alpha must not overlap the fields. */
iso_status iso_plan_run(iso_plan *plan, double *alpha, const double *phi, int64_t phi_stride, const double *U,
                        int64_t U_stride, double dt, int32_t n_steps);
/* Same step, also writing the intermediates named in trace (device pointers). */
iso_status iso_advect_step_traced(iso_plan *plan, const double *alpha, const double *phi, const double *U,
                                  double dt, double *alpha_new, iso_step_stats *stats, const iso_trace *trace);
/* The step of an outer (nonlinear) iteration, second order in time (Crank-Nicolson, end of
 * Section 3.2): the fluxes and velocities are the time averages (phi0 + phi1)/2 and (U0 + U1)/2
 * of the fields at t (phi0, U0) and the current estimates at t + dt (phi1, U1), formed as the
 * kernels read them (no averaged copy is written).  Layouts as iso_advect_step; all DEVICE arrays;
 * alpha_new must not overlap any input.  The result is bit for bit iso_advect_step with the
 * averaged fields.  For its adjoint, call iso_advect_step_adjoint with the averaged fields: each
 * level's phi_bar is then half the returned one. */
iso_status iso_advect_step_avg(iso_plan *plan, const double *alpha, const double *phi0, const double *phi1,
                               const double *U0, const double *U1, double dt, double *alpha_new,
                               iso_step_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the step of iso_advect_step without a plan, running the
 * same kernels, bit for bit the same alpha_new.  Its workspace is a fixed array of 64 MiB per
 * device inside the library, held from the first call on a device until the process ends; the call
 * allocates nothing.  Limit: about 24 B per cell plus 60 B per face (meshes of up to ~400k cells of
 * a 2D slab), ISO_ENOSPACE beyond.  mesh: created beforehand, on the current device; opt (nullable:
 * defaults) as for a plan, except check_inputs (ISO_EINVAL), max_surface (ignored: every cell fits)
 * and the statistics (none); stream: hipStream_t as void*, NULL = default stream.  alpha, phi, U,
 * alpha_new: DEVICE arrays laid out as for iso_advect_step.  Every call on one device shares that
 * device's workspace, whose contents the next call reuses: calls that overlap on one device (other
 * streams or threads) race and must be serialised by the caller. */
iso_status iso_advect_step_noalloc(const iso_mesh *mesh, const iso_options *opt, void *hip_stream,
                                   const double *alpha, const double *phi, const double *U, double dt,
                                   double *alpha_new);

/* Ghost-fluid face data after advection (Section 3.1, Eqs. 12-20): what the interface-corrected
 * interpolation of the dynamic pressure needs from the new volume fractions.  A cell is wet
 * (heavy fluid, density rho_heavy) iff alpha > 1/2.  For every face with a cell on each side (an
 * internal face, or the face of a cyclic pair that carries the flux, the partner's cell centre
 * moved into the owner's frame by the pair's translation) whose two cells are one wet and one dry:
 *   lambda    = (alpha_P - 1/2) / (alpha_P - alpha_N), P the face's owner (Eq. 13), and
 *               x_Gamma = x_P + lambda (x_N - x_P) (Eq. 12) from the cell centroids;
 *   jump      = p_d^- - p_d^+ at x_Gamma = (rho_heavy - rho_light) g . x_Gamma (the jump of Eq. 7,
 *               which Eq. 3 fixes for a continuous pressure; Eq. 15 prints the opposite sign);
 *   beta_w    = l / rho_light + (1 - l) / rho_heavy, l the distance fraction of x_Gamma from the wet
 *               cell (Eq. 18);
 *   ghost_nbr = p_d at the neighbour's centre seen from the owner's fluid, ghost_own = p_d at the
 *               owner's centre seen from the neighbour's fluid: the heavy fluid's value at the
 *               dry cell by Eq. 20, the light fluid's at the wet cell by the mirror expression.
 * Every other face: lambda = -1, jump = beta_w = 0, ghost_own = p_d of the owner, ghost_nbr = p_d
 * of the neighbour (of the owner where the face has one cell, and on the partner face of a
 * cyclic pair, which carries nothing of its own).
 * alpha, p_d [n_cells] (p_d: the dynamic pressure p - rho g . x per cell) and the five outputs
 * [n_faces] are DEVICE arrays; the outputs must not overlap the inputs or each other.
 * rho_heavy, rho_light > 0; g = (gx, gy, gz) the gravitational acceleration.  Asynchronous on the
 * plan's stream; nothing is allocated.  The arithmetic is rounded operation by operation in the
 * order written above (no fused multiply-add). */
iso_status iso_gfm_faces(iso_plan *plan, const double *alpha, const double *p_d, double rho_heavy,
                         double rho_light, double gx, double gy, double gz, double *lambda, double *jump,
                         double *beta_w, double *ghost_own, double *ghost_nbr);

/* Relaxation zones (Section 3, wave generation and absorption): after the advection step alpha
 * is blended explicitly towards a target solution (e.g. an incident wave's) with the exponential
 * weight of Jacobsen, Fuhrman & Fredsoe (2012), which the paper cites:
 *     alpha <- w alpha + (1 - w) alpha_target,   w(chi) = 1 - (exp(chi^3.5) - 1) / (e - 1),
 * chi = ((x_P - origin) . e) / length in [0, 1] for the cell centroid x_P, e = direction/|direction|:
 * w = 1 at the zone's inner edge (origin; the computed solution is kept), w = 0 at its outer edge
 * (the target is imposed).  A zone is the slab 0 <= chi <= 1; cells outside every zone are left
 * alone. */
typedef struct {
    double origin[3];     /* a point of the zone's inner edge */
    double direction[3];  /* into the zone, towards its outer edge (any non-zero length) */
    double length;        /* extent of the zone along direction (> 0) */
} iso_relax_zone;
/* Sets the plan's zones (host array, copied; n_zones = 0 clears them).  Finds the cells whose
 * centroids lie in a zone and their weights once, on the host, and keeps them on the device (12
 * bytes per zone cell; this call allocates, iso_relax_blend does not).  n_zone_cells (nullable)
 * receives their number.  ISO_EINVAL for a zero or non-finite direction, a length that is not
 * positive, or a cell inside two zones.  Synchronises the plan's stream. */
iso_status iso_plan_set_relaxation(iso_plan *plan, int32_t n_zones, const iso_relax_zone *zones,
                                   int64_t *n_zone_cells);
/* Blends alpha [n_cells] in place towards alpha_target [n_cells] in the plan's zones (DEVICE arrays,
 * not overlapping; only the zone cells are read or written).  Asynchronous on the plan's stream; a
 * plan without zones does nothing.  Rounded operation by operation as written (no fused
 * multiply-add). */
iso_status iso_relax_blend(iso_plan *plan, double *alpha, const double *alpha_target);

/* Adjoint of one step (vector-Jacobian product; differentiation is not part of the paper's
 * method).  Given alpha_new_bar = dL/d alpha_new for the step iso_advect_step(alpha, phi, U, dt)
 * -> alpha_new, writes alpha_bar = dL/d alpha [n_cells] and phi_bar = dL/d phi [n_faces] (zero on
 * faces that carry no flux and on the partner faces of cyclic pairs).  U and dt are held fixed.
 * The derivative follows the step exactly: the interface cells' isovalue moves with the volume
 * constraint of Section 3.2 (implicit function; at a jump of the sub-volume it is the vertex
 * value), the swept integrals (Eqs. tv .. intaplus) are differentiated through the isoface, and
 * the bounding sweeps are replayed and reversed; values that chopping or clamping moves by more
 * than 1e-14 have zero derivative (a smaller move only removes round-off and passes the
 * derivative), and a face with phi = 0 passes no derivative to phi.  Branches (interface cells,
 * upwind sides, wet vertices, bounding activity) are those of the given state.
 * fwd (nullable, DEVICE pointers): the intermediates of this same step from
 * iso_advect_step_traced with the same plan; vert_alpha, kind, iso, dV and alpha_raw are used.
 * NULL recomputes the forward step internally.  All arrays are DEVICE arrays; alpha_bar and
 * phi_bar must not overlap the inputs.  Asynchronous on the plan's stream.  The first call
 * allocates the adjoint workspace (about 380 + (48 + 16 W) S bytes per cell, for S bounding
 * sweeps and W flux slots per cell, 84 bytes per face and 800 per general polyhedron).  At most 31 bounding sweeps
 * (ISO_EUNSUPPORTED).  Every sum is taken in a fixed order (atomics only build work lists, whose
 * order changes no result): the same inputs give the same bits on every call. */
iso_status iso_advect_step_adjoint(iso_plan *plan, const double *alpha, const double *phi, const double *U,
                                   double dt, const iso_trace *fwd, const double *alpha_new_bar, double *alpha_bar,
                                   double *phi_bar);

/* Kernel timing (measurement support).  iso_plan_set_timing(plan, n) records HIP events on the
 * plan's stream around each of the step's kernels for the next n steps (0 disables; events are
 * created here, not in the step).  iso_plan_timing syncs the stream and returns, per kernel
 * (0 interface-cell list, 1 interface cells, 2 update, 3 bounding), the summed milliseconds over the
 * recorded steps, and the number of recorded steps; it then clears the record. */
iso_status iso_plan_set_timing(iso_plan *plan, int32_t max_steps);
iso_status iso_plan_timing(iso_plan *plan, double *kernel_ms /* [4] */, int32_t *n_steps);

/* ---- Ensembles ---------------------------------------------------------------------------
 * Many independent meshes advanced together (batched execution; not part of the paper's
 * method).  The members' device arrays are concatenated into one mesh, so each kernel of a step
 * is a single launch over all members, and a run of up to 256 steps is captured once as a HIP
 * graph and replayed while its arguments stay the same (longer runs are launched step by step).
 * Every member computes bit for bit what iso_advect_step computes on its own mesh with the same
 * options and time step.  The ensemble copies the member meshes: they may be destroyed after. */
typedef struct iso_batch iso_batch;

/* meshes [n] (each created on the current device); opt as for a plan (NULL = defaults);
 * hip_stream: the caller's stream (NULL = the null stream) that ensemble calls are ordered on. */
iso_status iso_batch_create(const iso_mesh *const *meshes, int32_t n, const iso_options *opt, void *hip_stream,
                            iso_batch **out);
void iso_batch_destroy(iso_batch *batch);
/* host out cell_off[n+1], face_off[n+1]: member d owns cells [cell_off[d], cell_off[d+1]) and
 * faces [face_off[d], face_off[d+1]) of the concatenated arrays. */
iso_status iso_batch_layout(const iso_batch *batch, int64_t *cell_off, int64_t *face_off);
/* n_steps steps of every member (Section 3.2 step, as iso_advect_step).  alpha: DEVICE [N], in/out,
 * concatenated by member.  phi: DEVICE, step s reads the F faces at phi + s*phi_stride; U: DEVICE,
 * step s reads U + s*U_stride, [3N] structure of arrays over the concatenated cells; a stride of 0
 * reuses the same fields every step.  dt: HOST [n], each member's time step.  Asynchronous: ordered
 * after the caller's earlier work on its stream, and later work on that stream waits for it.
 * alpha must not overlap the fields (ISO_EINVAL). */
iso_status iso_batch_advect(iso_batch *batch, double *alpha, const double *phi, int64_t phi_stride, const double *U,
                            int64_t U_stride, const double *dt, int32_t n_steps);
/* Launch shapes in use: cfg[0..3] = block_cells, surface_blocks, surface_waves, bound_blocks.
 * They never change a result. */
iso_status iso_batch_config(const iso_batch *batch, int32_t *cfg);
iso_status iso_batch_set_config(iso_batch *batch, const int32_t *cfg);
/* Autotuner: times n_trial steps of every candidate launch shape (coordinate search over the
 * interface kernel's register budget and work-group count, the per-cell block size and the
 * bounding grid) from state alpha with the fields phi, U of one step (alpha is not modified)
 * and keeps the fastest.  cache_path (nullable): text file of earlier choices keyed by the
 * ensemble's layout; a match skips the trials, a new choice is appended.  best_ms (nullable): the
 * chosen shape's ms per step.  Synchronous. */
iso_status iso_batch_tune(iso_batch *batch, const double *alpha, const double *phi, const double *U, const double *dt,
                          int32_t n_trial, const char *cache_path, double *best_ms);

#ifdef __cplusplus
}
#endif
#endif
