// Internal declarations shared by the host plan and the HIP kernels of the isoAdvector step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "isoadv.h"

namespace isoadv {

// A slot of a cell's flux list packs the flux-face id and the side of the cell:
// v >= 0: face v, phi > 0 leaves the cell; v < 0 (and not kEmpty): face ~v, phi > 0 enters it.
constexpr int32_t kEmpty = INT32_MIN;
__host__ __device__ inline int32_t pack_face(int32_t fid, int sign) { return sign > 0 ? fid : ~fid; }

// Canonical hexahedron: vertices 0-3 bottom loop, 4-7 above them; faces listed counter-clockwise
// seen from outside (bottom, top, y-, x+, y+, x- for an axis-aligned box).
constexpr int kHexFace[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
// Its edges (each with the end the cut computations start from first), and the edge under each
// face's loop position.
constexpr int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                              {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
constexpr int kFaceEdge[6][4] = {{3, 2, 1, 0}, {4, 5, 6, 7}, {0, 9, 4, 8}, {1, 10, 5, 9}, {2, 11, 6, 10}, {3, 8, 7, 11}};
// A face's loop as one word (bits 3i..3i+2 the vertex at loop position i, bit 12 a face, bit 16+i
// position i runs along its edge's direction): the canonical hexahedron's face k in the
// directions the hexahedron kernels take (kEdge).
constexpr int32_t hex_loop_word(int k) {
    int32_t w = 1 << 12;
    for (int i = 0; i < 4; ++i) {
        w |= kHexFace[k][i] << (3 * i);
        if (kEdge[kFaceEdge[k][i]][0] == kHexFace[k][i]) w |= 1 << (16 + i);
    }
    return w;
}

// Device view of a mesh, passed to kernels by value.
struct DevMesh {
    int32_t n_cells = 0, n_faces = 0, n_classes = 0, W = 0, n_patches = 0;
    const double *cxyz = nullptr;      // [24*n_cells] canonical vertex coordinates, cell-major
    const int32_t *cpt = nullptr;      // [8*n_cells] point class of each canonical vertex
    const double *vol = nullptr;       // [n_cells]
    const int32_t *slot_face = nullptr;  // [W][n_cells] packed flux faces, ascending face id, kEmpty last
    const int32_t *slot_nbr = nullptr;   // [W][n_cells] cell across the face, or -1-patch on the boundary
    // [n_cells][W] the same two tables cell-major, (slot_face, slot_nbr) per slot: the bounding
    // sweeps visit scattered cells, and find each one's slots in one run of 8 W bytes
    const int2 *slot_pair = nullptr;
    // [W][n_cells] the same slots in one 32-bit word each, which the update reads instead (null
    // when more than a tenth of the flux slots do not fit).  Upper half: the neighbour's offset from
    // the cell, positive offsets less one (an offset in [-32768, 32768] other than 0).  Lower half:
    // the face id less floor(owner * nar_S / 2^28), where the owner is the lower-numbered of the two
    // cells (which fixes the side) and nar_S = floor(n_internal 2^28 / n_cells).  0xFFFE: an empty
    // slot; 0xFFFF: read this slot from slot_face and slot_nbr (boundary faces, cyclic pairs, and
    // internal faces whose owner is the higher-numbered cell or whose offsets do not fit).
    const uint32_t *slot_nar = nullptr;
    uint32_t nar_S = 0;
    const int32_t *lface = nullptr;      // [6*n_cells] packed flux face of each canonical face, or kEmpty
    const int32_t *cflags = nullptr;     // [n_cells] bit k: canonical face k is planar
    const int32_t *st_ptr = nullptr;     // [n_classes+1] vertex stencils
    const int32_t *st_cell = nullptr;
    const double *st_w = nullptr;        // normalised inverse-distance weights
    const double *patch_alpha = nullptr; // [n_patches]
    const double *ccen = nullptr;        // [3*n_cells] cell centroids (same frame as cxyz), AoS
    // face-major table of the ghost-fluid face data (single meshes only; null in an ensemble)
    int32_t n_internal = 0;
    const int32_t *fcell = nullptr;      // [2*n_faces] owner, cell across (-1: none, or the partner
                                         // face of a cyclic pair)
    const int32_t *bpatch = nullptr;     // [n_faces-n_internal] patch of each boundary face
    const double *ptrans = nullptr;      // [3*n_patches] cyclic translations (x_partner = x + T)
    // local face loops of every cell (see plan.cpp), or null when every cell is a hexahedron
    const int32_t *cloop = nullptr;      // [6*n_cells]
    // general polyhedra (beyond 6 faces, 8 points or 4 points per face): null when there are none
    const int32_t *cbig = nullptr;       // [n_cells] index among them, or -1
    const int32_t *bv_ptr = nullptr;     // [n_big+1] points of each
    const int32_t *bv_cls = nullptr;     //   point class of each point
    const double *bv_xyz = nullptr;      //   its coordinates in the cell's frame
    const int32_t *bf_ptr = nullptr;     // [n_big+1] faces of each
    const int32_t *bf_face = nullptr;    //   packed flux face (kEmpty: none)
    const int32_t *bf_planar = nullptr;  //   1 if planar
    const int32_t *bl_ptr = nullptr;     // [faces+1] loop positions of each face
    const int32_t *bl_vtx = nullptr;     //   local point at each loop position, outward
    int32_t big_face_pts = 0;            // most points of a face of any of them
    int32_t all_big = 0;                 // 1: every cell is taken as one of them (mostly polyhedra)
    int32_t big_class = -1;              // 2: polyhedra of both instantiation classes (cflags bit
                                         // 11: the mesh they come from has faces of more than 4
                                         // points), each launch taking its own class
    // ensembles: cells [dom_off[d], dom_off[d+1]) belong to member d, whose time step is
    // dt_dom[d] (n_dom = 0 for a single mesh: one scalar time step)
    int32_t n_dom = 0;
    const int32_t *dom_off = nullptr;    // [n_dom+1]
    // ensembles: each member's words, as its own mesh has them (0xFFFF throughout for a member
    // without them), decoded with the member's nar_S,
    // first cell c0 and face offset f0 (face = f0 + floor((owner - c0) nar_S / 2^28) + low half).
    // [8 per 64 cells]: nar_S, f0, c0 of the member holding the block's first cell, the position
    // in the block where the next member starts (64: none; -1: more than two members meet there),
    // then nar_S, f0, c0 of that next member and the index of the first.  [3 n_dom]: nar_S, f0, c0
    // per member, for the blocks where more than two meet.
    const int32_t *nar_blk = nullptr;
    const int32_t *nar_dom = nullptr;
};

// Workspace of a plan (device pointers).
struct DevWork {
    int32_t *counters = nullptr;   // [kCntNum] see kCnt* below
    int32_t *surf = nullptr;       // [cap] interface cells
    double *dvs = nullptr;         // [n_faces] dV written by interface upwind cells
    int32_t *olist = nullptr;      // [n_cells] cells out of bounds after the update
    int32_t *tlist = nullptr;      // [2*n_cells] cells touched by a sweep (two banks by sweep parity)
    int32_t *flist = nullptr;      // [4*n_faces] faces whose dV changed during bounding; then the faces
                                   // holding a correction in each of the three correction buffers
    int32_t *cmark = nullptr;      // [2*n_cells] touched marks (two banks by sweep parity), zero between steps
    int32_t *fmark = nullptr;      // [n_faces] zero between steps
    double *delta = nullptr;       // [3*n_faces] correction buffers (sweep mod 3), zero between steps
    double *dvcur = nullptr;       // [n_faces] current dV of faces in flist
    double *red = nullptr;         // [kRedSize] statistics: the results, then per-work-group partial values
    double *sbnd = nullptr;        // [n_cells] volume through the cell's boundary faces (statistics only)
    double *sclip = nullptr;       // [n_cells] volume the chops added to the cell (statistics only)
    int32_t cap = 0;
    // meshes with general polyhedra: a second stream (default priority) for their interface
    // kernel, forked once the interface list is built and joined before the update, so that it
    // runs beside the eight-lane kernel
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

constexpr int kRedSize = 8 + 6 * 256;  // statistics reduction buffer (see launch_stats)

enum : int {
    kCntSurf = 0,       // interface cells found
    kCntOff = 1,        // cells needing redistribution (first list)
    kCntOverflow = 2,   // interface cells beyond capacity
    kCntFlat = 3,
    kCntNonconv = 4,
    kCntMaxIter = 5,
    kCntActive0 = 6,    // n_bound_active of the last step
    kCntFaces = 7,      // flist length
    kCntBound = 16,     // [16, 24): four rotating slots of per-sweep bounding counters
    kCntNum = 32
};

struct StepArgs {
    const double *alpha;
    const double *phi;
    const double *U;
    double *alpha_new;
    double dt;
    const double *dt_dom;  // [n_dom] per-member time steps of an ensemble, or nullptr
    // second time level of an outer iteration (or nullptr): the kernels read (phi + phi1)/2 and
    // (U + U1)/2
    const double *phi1 = nullptr;
    const double *U1 = nullptr;
};

// Launch shapes of a step (none of them changes a result).
struct LaunchCfg {
    int block_cells;    // threads per block of the per-cell kernels
    int surface_blocks; // work-groups of the interface kernel (0: from the list capacity)
    int surface_waves;  // register budget of the interface kernel, waves per SIMD (1-4)
    int bound_blocks;   // work-groups of the bounding sweeps
    int compact_slots;  // the update reads the mesh's 32-bit slot words where it has them
};

struct Params {
    double eps_surf, flat_tol, bound_tol;
    int32_t root_max_iter, n_bound_iter, clip;
    int32_t us_mode;  // 0: U_S = U_P; 1: cell-point interpolation to x_S
    double root_tol;  // isovalue search stops at |V_sub/V - alpha| <= root_tol (0: to round-off)
};

// Adjoint workspace (device pointers; allocated by a plan on its first adjoint step).  S = number of
// bounding sweeps (at least 1), nc cells, nf faces.
// adjoint counters: the interface cells' (cell, direction) pairs to differentiate along, then per
// sweep s the length of its list of
// cells out of bounds (kAdjL + s) and of the cells its corrections touch (kAdjT + s)
enum : int { kAdjDirs = 2, kAdjDirsBig = 3, kAdjGBig = 68, kAdjL = 8, kAdjT = 40, kAdjNum = 72, kAdjMaxSweeps = 31, kAdjG = 20,
             kAdjBoundBlocks = 512 };
struct AdjWork {
    int32_t *counters = nullptr;  // [kAdjNum]
    double *x = nullptr;          // [nc] bounding state
    double *xbar = nullptr;       // [nc] its adjoint
    double *pv = nullptr;         // [nc] adjoint of the update before its round-off chop, over the volume
    int32_t *cflag = nullptr;     // [nc] bit s: chopped or clamped in sweep s
    int32_t *list = nullptr;      // [S nc] cells listed in each sweep
    int32_t *tlist = nullptr;     // [S nc] cells touched in each sweep
    int32_t *cmark = nullptr;     // [2 nc] two banks of cell marks, zero between calls
    double *tape = nullptr;       // [S nc (4 + 2 W)]
    uint64_t *tflag = nullptr;    // [S nc]
    double *dvcur = nullptr;      // [nf] running dV of corrected faces
    int32_t *touched = nullptr;   // [nf] faces corrected in an earlier sweep, zero between calls
    double *delta = nullptr;      // [3 nf] three rotating correction buffers, zero between calls
    double *dVb = nullptr;        // [nf] adjoint of dV before bounding, from bounding
    double *phib = nullptr;       // [nf] adjoint of phi, from bounding
    double *dvcurbar = nullptr;   // [nf]
    double *deltabar = nullptr;   // [nf]
    double *vbar = nullptr;       // [nf] adjoint of the swept integral of interface-upwind faces, times phi
    double *gbuf = nullptr;       // [kAdjG nc] reconstructed cells: rates along their 8 vertex values and the
                                  // isovalue (see adjoint.hip)
    double *pbar = nullptr;       // [n_classes] adjoint of each point class's vertex value
    int64_t *dlist = nullptr;     // [9 nc] (cell << 4 | direction) pairs of the interface cells
    // general polyhedra: (cell << 6 | direction) pairs, and the rates per polyhedron
    int64_t *dlist_big = nullptr;  // [33 n_big]
    double *gbig = nullptr;        // [kAdjGBig n_big]
    int32_t big_cap = 0;           // n_big
};
struct AdjInputs {
    const double *vert_alpha;  // forward intermediates of the step
    const int32_t *kind;
    const double *iso;
    const double *dV;
    const double *raw;
    const double *abar_new;    // adjoint in
    double *abar, *phibar;     // adjoints out
};

// kernels.hip
// ev: nullptr, or 5 events recorded before each of the 4 kernels and after the last
hipError_t launch_step(const DevMesh &m, const DevWork &w, const Params &p, const StepArgs &a,
                       const iso_trace *trace, const LaunchCfg &cfg, bool want_stats, hipStream_t s, hipEvent_t *ev);
// dst[i] = src[i] with offsets (ensemble meshes).  mode 0: v >= 0 -> v + off1;  mode 1 (packed flux
// face): kEmpty kept, v >= 0 -> v + off1, else ~(~v + off1);  mode 2 (cell across a face): v >= 0 ->
// v + off1, else -1 - (-1 - v + off2).  src == nullptr fills dst with off1.
hipError_t launch_offset_copy(const int32_t *src, int32_t *dst, int64_t n, int mode, int32_t off1, int32_t off2,
                              hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);
// m.slot_pair from m.slot_face and m.slot_nbr (pairs: [n_cells * W] device array)
hipError_t launch_slot_pairs(const DevMesh &m, int2 *pairs, hipStream_t s);
// adjoint.hip
hipError_t launch_adjoint(const DevMesh &m, const Params &p, const StepArgs &a, const AdjInputs &in, const AdjWork &w,
                          hipStream_t s);
// General polyhedra: limits of their sixteen-lanes-per-cell interface kernel (big.hip).
constexpr int kBigPts = 32, kBigFaces = 16, kBigFacePts = 16;
struct BigArgs {
    DevMesh m;
    const double *alpha, *phi, *U;
    const double *phi1, *U1;  // second time level of an outer iteration, or nullptr
    double dt, flat_tol;
    int max_rounds;
    const double *dt_dom;     // ensembles: each member's time step (see DevMesh::n_dom), else nullptr
    const int32_t *list;
    int32_t *counters;
    int cap;
    double *dvs;
    int want_stats;
    iso_trace tr;
    double root_tol;  // as Params::root_tol
    int us_mode;      // as Params::us_mode
    int only_class = -1;  // >= 0: only polyhedra of this instantiation class (cflags bit 11)
};
hipError_t launch_surface_big(const BigArgs &a, hipStream_t s);

// Ghost-fluid face data (Eqs. 12-20): see gfm.hip.
struct GfmArgs {
    const int32_t *fcell, *bpatch;
    const double *ptrans, *ccen;
    const double *alpha, *p_d;
    double *lambda, *jump, *beta_w, *ghost_own, *ghost_nbr;
    double b_heavy, b_light, drho;  // 1/rho^+, 1/rho^-, rho^+ - rho^-
    double g[3];
    int64_t n_faces;
    int32_t n_internal;
};
hipError_t launch_gfm_faces(const GfmArgs &a, hipStream_t s);
// Relaxation-zone blend (relax.hip): alpha[cells[i]] = w[i] alpha + (1 - w[i]) target, in place.
hipError_t launch_relax_blend(const int32_t *cells, const double *w, int64_t n, double *alpha, const double *target,
                              hipStream_t s);
hipError_t launch_stats(const DevMesh &m, const DevWork &w, const double *alpha, const double *alpha_new,
                        hipStream_t s);

}  // namespace isoadv

struct iso_mesh {
    isoadv::DevMesh dev;
    int32_t n_points = 0, n_faces = 0, n_internal = 0, n_cells = 0, n_flux = 0, n_classes = 0, W = 0;
    std::vector<int32_t> cell_pts;   // [8*n_cells] user point ids, canonical order (a cell with fewer
                                     // points repeats its first one after them)
    std::vector<int32_t> nvtx;       // [n_cells] distinct points of each cell
    bool generic = false;            // some cell is not a hexahedron
    // general polyhedra: how many, and the lengths of their point, face and loop arrays
    int32_t n_big = 0, n_bv = 0, n_bf = 0, n_bl = 0;
    int64_t n_wide_slots = -1;       // flux slots the 32-bit words send to the full tables (-1: no words)
    std::vector<double> vol, xc;
    std::vector<double> patch_alpha;
    int64_t st_nnz = 0;              // entries of the vertex stencils
    std::vector<void *> allocations;
    int64_t device_bytes = 0;
    int device = 0;
};

struct iso_plan {
    const iso_mesh *mesh = nullptr;
    iso_options opt{};
    hipStream_t stream = nullptr;
    isoadv::DevWork work;
    std::vector<void *> allocations;
    int32_t *host_counters = nullptr;  // pinned [kCntNum]
    double *host_red = nullptr;        // pinned [64]
    std::vector<hipEvent_t> events;    // 5 per recorded step
    int32_t timing_cap = 0, timing_used = 0;
    // adjoint workspace and forward-trace buffers (allocated on the first adjoint step)
    isoadv::AdjWork adj;
    double *adj_vert = nullptr, *adj_iso = nullptr, *adj_dV = nullptr, *adj_raw = nullptr, *adj_new = nullptr;
    int32_t *adj_kind = nullptr;
    bool adj_ready = false;
    // relaxation zones (iso_plan_set_relaxation): zone cells and their weights
    int32_t *rz_cell = nullptr;
    double *rz_w = nullptr;
    int64_t rz_n = 0;
    // multi-step runs (iso_plan_run): the second state buffer (allocated on the first run), the
    // run's own stream with the events that order it after and before the plan's stream, and the
    // captured graph of the last run with the arguments it was captured for
    double *run_tmp = nullptr;
    hipStream_t run_stream = nullptr;
    hipEvent_t run_in = nullptr, run_out = nullptr;
    hipGraph_t run_graph = nullptr;
    hipGraphExec_t run_exec = nullptr;
    struct RunKey {
        double *alpha = nullptr;
        const double *phi = nullptr, *U = nullptr;
        int64_t ps = 0, us = 0;
        double dt = 0.0;
        int32_t steps = 0;
    } run_key;
    bool run_have = false;
};

namespace isoadv {
iso_status fail(iso_status s, const std::string &msg);
LaunchCfg launch_cfg(const iso_options &o);
Params step_params(const iso_options &o);
// option ranges, and what the mesh's cells support (ISO_EINVAL, ISO_EUNSUPPORTED)
iso_status check_options(const iso_options &o, const iso_mesh *mesh);
// non-null arrays, dt > 0 and finite, alpha_new overlapping no input (ISO_EINVAL)
iso_status check_step_args(const iso_mesh *m, const double *alpha, const double *phi, const double *U, double dt,
                           double *alpha_new, const double *phi1, const double *U1);
}
