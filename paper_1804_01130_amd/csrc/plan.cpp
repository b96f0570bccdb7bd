// Host side of the isoAdvector library: mesh validation and device layout, plans, and the
// C entry points.  Geometry follows Section 3 of the paper (collocated polyhedral cells with
// owner/neighbour faces); the per-step work is in kernels.hip.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace isoadv;

namespace {

thread_local std::string g_last_error;

struct V3 {
    double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

template <class T>
iso_status upload(iso_mesh *m, const std::vector<T> &h, const T **dptr) {
    void *p = nullptr;
    size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(ISO_ENOMEM, "hipMalloc failed for mesh array");
    m->allocations.push_back(p);
    m->device_bytes += (int64_t)bytes;
    if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(ISO_EDEVICE, "hipMemcpy failed for mesh array");
    *dptr = static_cast<const T *>(p);
    return ISO_OK;
}

// weighted union-find over points: x_p + off[p] is p's position in the frame of parent[p]
struct FrameUnion {
    std::vector<int32_t> parent;
    std::vector<V3> off;
    explicit FrameUnion(int n) : parent(n), off(n, V3{0, 0, 0}) { std::iota(parent.begin(), parent.end(), 0); }
    int32_t find(int32_t p, V3 *to_root) {
        V3 acc{0, 0, 0};
        int32_t r = p;
        while (parent[r] != r) {
            acc = acc + off[r];
            r = parent[r];
        }
        // compress
        V3 run = acc;
        int32_t q = p;
        while (parent[q] != q) {
            int32_t nx = parent[q];
            V3 oq = off[q];
            parent[q] = r;
            off[q] = run;
            run = run - oq;
            q = nx;
        }
        *to_root = acc;
        return r;
    }
    // x_b = x_a + T (same physical point seen from two frames)
    bool unite(int32_t a, int32_t b, V3 T) {
        V3 da, db;
        int32_t ra = find(a, &da), rb = find(b, &db);
        if (ra == rb) return true;
        // frame ra -> frame a: -da; frame a -> frame b: +T; frame b -> frame rb: +db
        parent[ra] = rb;
        off[ra] = T + db - da;
        return true;
    }
};

}  // namespace

namespace isoadv {
iso_status fail(iso_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}
LaunchCfg launch_cfg(const iso_options &o) {
    LaunchCfg c;
    c.block_cells = o.block_cells > 0 ? o.block_cells : 256;
    c.surface_blocks = o.surface_blocks;
    c.surface_waves = o.surface_waves > 0 ? o.surface_waves : 2;
    c.bound_blocks = o.bound_blocks > 0 ? o.bound_blocks : 512;
    c.compact_slots = o.full_slots ? 0 : 1;
    return c;
}
Params step_params(const iso_options &o) {
    return Params{o.eps_surf, o.flat_tol, o.bound_tol, o.root_max_iter, o.n_bound_iter, o.clip, o.us_mode, o.root_tol};
}
iso_status check_options(const iso_options &o, const iso_mesh *mesh) {
    if (!(o.eps_surf >= 0 && o.eps_surf < 0.5) || !(o.flat_tol >= 0) || !(o.bound_tol >= 0) || o.root_max_iter < 1 ||
        o.n_bound_iter < 0 || o.block_cells < 0 || o.block_cells > 1024 ||
        o.surface_blocks < 0 || o.surface_blocks > 65535 || o.bound_blocks < 0 || o.bound_blocks > 65535 ||
        o.max_surface < 0 || o.surface_waves < 0 || o.surface_waves > 4 || o.us_mode < 0 || o.us_mode > 1 ||
        !(o.root_tol >= 0 && o.root_tol < 1) || o.full_slots < 0 || o.full_slots > 1)
        return fail(ISO_EINVAL, "bad options");
    return ISO_OK;
}
static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}
iso_status check_step_args(const iso_mesh *m, const double *alpha, const double *phi, const double *U, double dt,
                           double *alpha_new, const double *phi1, const double *U1) {
    if (!alpha || !phi || !U || !alpha_new) return fail(ISO_EINVAL, "null array");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(ISO_EINVAL, "dt must be positive and finite");
    size_t nc = (size_t)m->n_cells * 8, nf = (size_t)m->n_faces * 8;
    if (overlaps(alpha_new, nc, alpha, nc) || overlaps(alpha_new, nc, phi, nf) || overlaps(alpha_new, nc, U, 3 * nc) ||
        (phi1 && overlaps(alpha_new, nc, phi1, nf)) || (U1 && overlaps(alpha_new, nc, U1, 3 * nc)))
        return fail(ISO_EINVAL, "alpha_new overlaps an input");
    return ISO_OK;
}
}  // namespace isoadv

extern "C" {

const char *iso_last_error(void) { return g_last_error.c_str(); }

const char *iso_status_string(iso_status s) {
    switch (s) {
        case ISO_OK: return "ok";
        case ISO_EINVAL: return "invalid argument";
        case ISO_ENOMEM: return "out of memory";
        case ISO_EDEVICE: return "device error";
        case ISO_ENOSPACE: return "interface-cell capacity exceeded";
        case ISO_ECOURANT: return "Courant number above limit";
        case ISO_EMESH: return "inconsistent mesh";
        case ISO_EUNSUPPORTED: return "unsupported cell type";
    }
    return "unknown status";
}

void iso_options_default(iso_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps_surf = 1e-8;
    o->flat_tol = 1e-12;
    o->bound_tol = 1e-12;
    o->max_courant = 1.0;
    o->root_max_iter = 100;
    o->n_bound_iter = 3;
    o->clip = 1;
}

void iso_mesh_destroy(iso_mesh *m) {
    if (!m) return;
    for (void *p : m->allocations) (void)hipFree(p);
    delete m;
}

iso_status iso_mesh_create(int32_t n_points, const double *px, const double *py, const double *pz, int32_t n_faces,
                           const int32_t *face_ptr, const int32_t *face_pts, const int32_t *owner,
                           int32_t n_internal, const int32_t *neighbour, int32_t n_cells, int32_t n_patches,
                           const int32_t *patch_start, const int32_t *patch_size, const int32_t *patch_kind,
                           const int32_t *patch_partner, const double *patch_translation,
                           const double *patch_alpha_in, iso_mesh **out) {
    if (!out) return fail(ISO_EINVAL, "out is null");
    *out = nullptr;
    if (n_points <= 0 || n_faces <= 0 || n_cells <= 0 || n_internal < 0 || n_internal > n_faces || n_patches < 0)
        return fail(ISO_EINVAL, "bad mesh sizes");
    if (!px || !py || !pz || !face_ptr || !face_pts || !owner || (n_internal > 0 && !neighbour))
        return fail(ISO_EINVAL, "null mesh array");
    if (n_patches > 0 && (!patch_start || !patch_size || !patch_kind || !patch_partner || !patch_translation ||
                          !patch_alpha_in))
        return fail(ISO_EINVAL, "null patch array");

    // ---- connectivity checks
    if (face_ptr[0] != 0) return fail(ISO_EMESH, "face_ptr[0] != 0");
    for (int32_t f = 0; f < n_faces; ++f) {
        if (face_ptr[f + 1] < face_ptr[f]) return fail(ISO_EMESH, "face_ptr not monotone");
        if (owner[f] < 0 || owner[f] >= n_cells) return fail(ISO_EMESH, "owner out of range at face " + std::to_string(f));
    }
    for (int32_t k = 0; k < face_ptr[n_faces]; ++k)
        if (face_pts[k] < 0 || face_pts[k] >= n_points) return fail(ISO_EMESH, "face point out of range");
    for (int32_t f = 0; f < n_internal; ++f)
        if (neighbour[f] < 0 || neighbour[f] >= n_cells || neighbour[f] == owner[f])
            return fail(ISO_EMESH, "neighbour out of range at face " + std::to_string(f));
    std::vector<int32_t> fpatch(n_faces, -1);
    for (int32_t p = 0; p < n_patches; ++p) {
        if (patch_start[p] < n_internal || patch_size[p] < 0 || patch_start[p] + patch_size[p] > n_faces)
            return fail(ISO_EMESH, "patch range out of the boundary faces");
        if (patch_kind[p] < ISO_PATCH_WALL || patch_kind[p] > ISO_PATCH_CYCLIC) return fail(ISO_EMESH, "bad patch kind");
        for (int32_t f = patch_start[p]; f < patch_start[p] + patch_size[p]; ++f) {
            if (fpatch[f] >= 0) return fail(ISO_EMESH, "patches overlap");
            fpatch[f] = p;
        }
        if (patch_kind[p] == ISO_PATCH_CYCLIC) {
            int32_t q = patch_partner[p];
            if (q < 0 || q >= n_patches || q == p || patch_kind[q] != ISO_PATCH_CYCLIC || patch_partner[q] != p ||
                patch_size[q] != patch_size[p])
                return fail(ISO_EMESH, "cyclic patch " + std::to_string(p) + " has no matching partner");
        }
    }
    for (int32_t f = n_internal; f < n_faces; ++f)
        if (fpatch[f] < 0) return fail(ISO_EMESH, "boundary face " + std::to_string(f) + " in no patch");

    auto P = [&](int32_t i) { return V3{px[i], py[i], pz[i]}; };

    // ---- cells: hexahedra (six quadrilaterals, the canonical vertex order below); other cells of
    // at most six faces of three or four points and at most eight distinct points (tetrahedra,
    // pyramids, prisms), whose faces are listed with their own vertex loops; and general polyhedra
    // up to kBigFaces faces of up to kBigFacePts points over up to kBigPts points
    std::vector<int32_t> ncf(n_cells, 0);
    for (int32_t f = 0; f < n_faces; ++f) {
        ncf[owner[f]]++;
        if (f < n_internal) ncf[neighbour[f]]++;
    }
    for (int32_t c = 0; c < n_cells; ++c)
        if (ncf[c] < 4 || ncf[c] > kBigFaces)
            return fail(ISO_EUNSUPPORTED, "cell " + std::to_string(c) + " has " + std::to_string(ncf[c]) +
                                              " faces (4 to " + std::to_string(kBigFaces) + " are taken)");
    for (int32_t f = 0; f < n_faces; ++f) {
        const int32_t np = face_ptr[f + 1] - face_ptr[f];
        if (np < 3 || np > kBigFacePts)
            return fail(ISO_EUNSUPPORTED, "face " + std::to_string(f) + " has " + std::to_string(np) +
                                              " points (3 to " + std::to_string(kBigFacePts) + " are taken)");
    }
    std::vector<int32_t> cf_ptr(n_cells + 1, 0);
    for (int32_t c = 0; c < n_cells; ++c) cf_ptr[c + 1] = cf_ptr[c] + ncf[c];
    std::vector<int32_t> cf_list(cf_ptr[n_cells], -1);
    std::fill(ncf.begin(), ncf.end(), 0);
    for (int32_t f = 0; f < n_faces; ++f) {  // ascending face id per cell
        cf_list[cf_ptr[owner[f]] + ncf[owner[f]]++] = f;
        if (f < n_internal) cf_list[cf_ptr[neighbour[f]] + ncf[neighbour[f]]++] = f;
    }
    auto cface = [&](int32_t c, int k) { return cf_list[cf_ptr[c] + k]; };
    // a face's points counter-clockwise seen from outside cell c (a triangle repeats its first point)
    auto outward = [&](int32_t f, int32_t c, std::array<int32_t, 4> &q) {
        const int32_t *fp = face_pts + face_ptr[f];
        const int np = face_ptr[f + 1] - face_ptr[f];
        if (owner[f] == c) for (int i = 0; i < np; ++i) q[i] = fp[i];
        else for (int i = 0; i < np; ++i) q[i] = fp[np - 1 - i];
        if (np == 3) q[3] = q[0];
    };
    auto npts = [&](int32_t f) { return face_ptr[f + 1] - face_ptr[f]; };
    // any face's points counter-clockwise seen from outside cell c
    auto outward_n = [&](int32_t f, int32_t c, int32_t *q) {
        const int32_t *fp = face_pts + face_ptr[f];
        const int np = npts(f);
        if (owner[f] == c) for (int i = 0; i < np; ++i) q[i] = fp[i];
        else for (int i = 0; i < np; ++i) q[i] = fp[np - 1 - i];
    };

    iso_mesh *m = new iso_mesh();
    m->n_points = n_points; m->n_faces = n_faces; m->n_internal = n_internal; m->n_cells = n_cells;
    m->cell_pts.resize(8 * (size_t)n_cells);
    m->nvtx.assign(n_cells, 8);
    std::vector<int32_t> lface_actual(6 * (size_t)n_cells, -1);
    // other cells: local vertex loop of each face (local indices 0-7, a triangle's fourth entry
    // repeating its first) and the number of points of the face (0: no face)
    std::vector<std::array<int8_t, 4>> gloop(6 * (size_t)n_cells, std::array<int8_t, 4>{0, 0, 0, 0});
    std::vector<int8_t> gnp(6 * (size_t)n_cells, 0);

    bool closed_ok = true;
    auto make_generic = [&](int32_t c) -> bool {
        // generic cell: distinct points in order of first appearance
        int32_t v[8];
        int nv = 0;
        bool ok = true;
        for (int k = 0; k < ncf[c] && ok; ++k) {
            std::array<int32_t, 4> q;
            const int32_t f = cface(c, k);
            outward(f, c, q);
            for (int i = 0; i < npts(f) && ok; ++i) {
                int j = 0;
                while (j < nv && v[j] != q[i]) ++j;
                if (j == nv) {
                    if (nv == 8) ok = false;
                    else v[nv++] = q[i];
                }
                gloop[6 * (size_t)c + k][i] = (int8_t)j;
            }
            if (npts(f) == 3) gloop[6 * (size_t)c + k][3] = gloop[6 * (size_t)c + k][0];
            gnp[6 * (size_t)c + k] = (int8_t)npts(f);
            lface_actual[6 * (size_t)c + k] = f;
        }
        if (!ok || nv < 4) {  // more than eight points (or a degenerate cell): leave nothing behind
            for (int k = 0; k < 6; ++k) { gnp[6 * (size_t)c + k] = 0; lface_actual[6 * (size_t)c + k] = -1; }
            return false;
        }
        for (int i = 0; i < 8; ++i) m->cell_pts[8 * (size_t)c + i] = v[i < nv ? i : 0];
        // closed: the outward area vectors of the faces sum to zero
        V3 sum{0, 0, 0};
        double mag = 0;
        for (int k = 0; k < ncf[c]; ++k) {
            std::array<int32_t, 4> q;
            const int32_t f = cface(c, k);
            outward(f, c, q);
            const V3 a = 0.5 * cross(P(q[2]) - P(q[0]), P(q[3]) - P(q[1]));
            sum = sum + a;
            mag += norm(a);
        }
        if (!(norm(sum) <= 1e-9 * mag)) closed_ok = false;
        m->nvtx[c] = nv;
        m->generic = true;
        return true;
    };

    // general polyhedra: their distinct points, and each face's loop of local point indices
    std::vector<int32_t> cbig(n_cells, -1), bv_ptr{0}, bv_pts, bf_ptr{0}, bf_fid, bl_ptr{0}, bl_vtx;
    auto make_big = [&](int32_t c) -> bool {
        std::vector<int32_t> v;
        int32_t q[kBigFacePts];
        for (int k = 0; k < ncf[c]; ++k) {
            const int32_t f = cface(c, k);
            outward_n(f, c, q);
            for (int i = 0; i < npts(f); ++i) {
                int j = 0;
                while (j < (int)v.size() && v[j] != q[i]) ++j;
                if (j == (int)v.size()) {
                    if ((int)v.size() == kBigPts) return false;
                    v.push_back(q[i]);
                }
                bl_vtx.push_back(j);
            }
            bl_ptr.push_back((int32_t)bl_vtx.size());
            bf_fid.push_back(f);
        }
        cbig[c] = (int32_t)bv_ptr.size() - 1;
        bv_pts.insert(bv_pts.end(), v.begin(), v.end());
        bv_ptr.push_back((int32_t)bv_pts.size());
        bf_ptr.push_back((int32_t)bf_fid.size());
        for (int i = 0; i < 8; ++i) m->cell_pts[8 * (size_t)c + i] = v[i < (int)v.size() ? i : 0];
        m->nvtx[c] = 0;  // the stencils take the points from the lists above
        m->generic = true;
        // closed: the outward area vectors of the faces sum to zero (Newell's area vector)
        V3 sum{0, 0, 0};
        double mag = 0;
        for (int k = 0; k < ncf[c]; ++k) {
            const int32_t f = cface(c, k);
            outward_n(f, c, q);
            V3 a{0, 0, 0};
            for (int i = 0; i < npts(f); ++i) a = a + 0.5 * cross(P(q[i]), P(q[(i + 1) % npts(f)]));
            sum = sum + a;
            mag += norm(a);
        }
        if (!(norm(sum) <= 1e-9 * mag)) closed_ok = false;
        return true;
    };

    for (int32_t c = 0; c < n_cells; ++c) {
        bool small = ncf[c] <= 6;
        for (int k = 0; k < ncf[c] && small; ++k) small = npts(cface(c, k)) <= 4;
        if (!small) {
            if (!make_big(c)) {
                iso_mesh_destroy(m);
                return fail(ISO_EUNSUPPORTED, "cell " + std::to_string(c) + " has more than " +
                                                  std::to_string(kBigPts) + " points");
            }
            continue;
        }
        bool hex = ncf[c] == 6;
        for (int k = 0; k < ncf[c] && hex; ++k) hex = npts(cface(c, k)) == 4;
        if (!hex) {
            if (!make_generic(c) && !make_big(c)) {
                iso_mesh_destroy(m);
                return fail(ISO_EUNSUPPORTED, "cell " + std::to_string(c) + " has more than " +
                                                  std::to_string(kBigPts) + " points or fewer than 4");
            }
            continue;
        }
        std::array<std::array<int32_t, 4>, 6> fq;
        for (int k = 0; k < 6; ++k) outward(cface(c, k), c, fq[k]);
        // bottom = first face; its outward loop is canonical (0,3,2,1)
        int32_t v[8];
        v[0] = fq[0][0]; v[3] = fq[0][1]; v[2] = fq[0][2]; v[1] = fq[0][3];
        // vertex above each bottom vertex: the one joined to it by an edge not on the bottom face
        auto on_bottom = [&](int32_t p) { return p == v[0] || p == v[1] || p == v[2] || p == v[3]; };
        bool ok = true;
        for (int b = 0; b < 4 && ok; ++b) {
            int32_t above = -1;
            for (int k = 1; k < 6; ++k)
                for (int i = 0; i < 4; ++i) {
                    int32_t a = fq[k][i], bb = fq[k][(i + 1) % 4];
                    int32_t other = a == v[b] ? bb : (bb == v[b] ? a : -1);
                    if (other >= 0 && !on_bottom(other)) {
                        if (above >= 0 && above != other) ok = false;
                        above = other;
                    }
                }
            if (above < 0) ok = false;
            v[4 + b] = above;
        }
        if (ok) {
            int32_t s[8];
            std::copy(v, v + 8, s);
            std::sort(s, s + 8);
            ok = std::adjacent_find(s, s + 8) == s + 8;
        }
        if (!ok) {  // six quadrilaterals that do not make a hexahedron
            if (!make_generic(c) && !make_big(c)) {
                iso_mesh_destroy(m);
                return fail(ISO_EUNSUPPORTED, "cell " + std::to_string(c) + " has more than " +
                                                  std::to_string(kBigPts) + " points or fewer than 4");
            }
            continue;
        }
        // match canonical faces to actual faces, with orientation
        for (int k = 0; k < 6; ++k) {
            int found = -1;
            for (int j = 0; j < 6 && found < 0; ++j) {
                for (int r = 0; r < 4; ++r) {
                    bool same = true;
                    for (int i = 0; i < 4; ++i) same = same && fq[j][(i + r) % 4] == v[kHexFace[k][i]];
                    if (same) { found = j; break; }
                }
            }
            if (found < 0) {
                iso_mesh_destroy(m);
                return fail(ISO_EMESH, "cell " + std::to_string(c) + ": faces inconsistently oriented");
            }
            lface_actual[6 * (size_t)c + k] = cface(c, found);
        }
        for (int i = 0; i < 8; ++i) m->cell_pts[8 * (size_t)c + i] = v[i];
    }

    // a mesh that is mostly general polyhedra runs every cell through their kernel (one launch, no
    // second stream): the other cells are taken as polyhedra of their own faces too
    bool all_big = false;
    {
        int64_t nbig = 0;
        for (int32_t c = 0; c < n_cells; ++c) nbig += cbig[c] >= 0 ? 1 : 0;
        if (nbig > 0 && 2 * nbig >= n_cells) {
            for (int32_t c = 0; c < n_cells; ++c)
                if (cbig[c] < 0 && !make_big(c)) {
                    iso_mesh_destroy(m);
                    return fail(ISO_EUNSUPPORTED, "cell " + std::to_string(c) + " has more than " +
                                                      std::to_string(kBigPts) + " points");
                }
            all_big = true;
        }
    }
    if (!closed_ok) { iso_mesh_destroy(m); return fail(ISO_EMESH, "a cell's faces do not close it"); }

    // ---- volumes and centroids: tetrahedra (vertex mean, face vertex mean, edge) over outward faces
    m->vol.resize(n_cells);
    m->xc.resize(3 * (size_t)n_cells);
    for (int32_t c = 0; c < n_cells; ++c) {
        if (cbig[c] >= 0) {
            // general polyhedron: the same pyramid decomposition over its point list and face loops
            const int b = cbig[c];
            const int32_t *v = &bv_pts[bv_ptr[b]];
            const int nv = bv_ptr[b + 1] - bv_ptr[b];
            V3 xm{0, 0, 0};
            for (int i = 0; i < nv; ++i) xm = xm + P(v[i]);
            xm = (1.0 / nv) * xm;
            double vol = 0;
            V3 mom{0, 0, 0};
            for (int k = bf_ptr[b]; k < bf_ptr[b + 1]; ++k) {
                const int l0 = bl_ptr[k], np = bl_ptr[k + 1] - l0;
                V3 ap{0, 0, 0};
                for (int i = 0; i < np; ++i) ap = ap + P(v[bl_vtx[l0 + i]]);
                ap = (1.0 / np) * ap;
                for (int i = 0; i < np; ++i) {
                    const V3 qi = P(v[bl_vtx[l0 + i]]), qj = P(v[bl_vtx[l0 + (i + 1) % np]]);
                    V3 a = ap - xm, bb = qi - xm, cc = qj - xm;
                    double tv = dot(a, cross(bb, cc)) / 6.0;
                    vol += tv;
                    mom = mom + (tv * 0.25) * (xm + ap + qi + qj);
                }
            }
            if (!(vol > 0)) { iso_mesh_destroy(m); return fail(ISO_EMESH, "cell " + std::to_string(c) + " has non-positive volume"); }
            m->vol[c] = vol;
            V3 x = (1.0 / vol) * mom;
            m->xc[3 * c] = x.x; m->xc[3 * c + 1] = x.y; m->xc[3 * c + 2] = x.z;
            continue;
        }
        const int32_t *v = &m->cell_pts[8 * (size_t)c];
        const int nv = m->nvtx[c];
        V3 xm{0, 0, 0};
        for (int i = 0; i < nv; ++i) xm = xm + P(v[i]);
        xm = (nv == 8 ? 0.125 : 1.0 / nv) * xm;
        double vol = 0;
        V3 mom{0, 0, 0};
        for (int k = 0; k < 6; ++k) {
            V3 q[4];
            int np = 4;
            if (gnp[6 * (size_t)c] == 0) {
                for (int i = 0; i < 4; ++i) q[i] = P(v[kHexFace[k][i]]);
            } else {
                np = gnp[6 * (size_t)c + k];
                if (np == 0) continue;
                for (int i = 0; i < np; ++i) q[i] = P(v[gloop[6 * (size_t)c + k][i]]);
            }
            V3 ap = np == 4 ? 0.25 * (q[0] + q[1] + q[2] + q[3]) : (1.0 / 3.0) * (q[0] + q[1] + q[2]);
            for (int i = 0; i < np; ++i) {
                V3 a = ap - xm, b = q[i] - xm, cc = q[(i + 1) % np] - xm;
                double tv = dot(a, cross(b, cc)) / 6.0;
                vol += tv;
                mom = mom + (tv * 0.25) * (xm + ap + q[i] + q[(i + 1) % np]);
            }
        }
        if (!(vol > 0)) { iso_mesh_destroy(m); return fail(ISO_EMESH, "cell " + std::to_string(c) + " has non-positive volume"); }
        m->vol[c] = vol;
        V3 x = (1.0 / vol) * mom;
        m->xc[3 * c] = x.x; m->xc[3 * c + 1] = x.y; m->xc[3 * c + 2] = x.z;
    }

    // ---- flux faces: interior, cyclic pairs (lower patch index carries phi), inflow/outflow
    // per (face): fid, sign seen from the face's owner, cell across (or -1-patch)
    std::vector<int32_t> f_fid(n_faces, -1), f_sign(n_faces, 0), f_other(n_faces, -1);
    int32_t n_flux = 0;
    for (int32_t f = 0; f < n_faces; ++f) {
        if (f < n_internal) { f_fid[f] = f; f_sign[f] = 1; f_other[f] = neighbour[f]; ++n_flux; continue; }
        int32_t p = fpatch[f];
        if (patch_kind[p] == ISO_PATCH_INOUT) { f_fid[f] = f; f_sign[f] = 1; f_other[f] = -1 - p; ++n_flux; }
        else if (patch_kind[p] == ISO_PATCH_CYCLIC) {
            int32_t q = patch_partner[p];
            int32_t g = patch_start[q] + (f - patch_start[p]);
            int32_t primary = p < q ? f : g;
            f_fid[f] = primary;
            f_sign[f] = primary == f ? 1 : -1;
            f_other[f] = owner[g];
            if (primary == f) ++n_flux;
        }
    }
    m->n_flux = n_flux;
    // face-major table of the ghost-fluid face data: owner and the cell across (the partner face's
    // owner for the face of a cyclic pair that carries the flux, -1 for every other boundary face)
    std::vector<int32_t> fcell(2 * (size_t)n_faces), bpatch(std::max(1, n_faces - n_internal));
    for (int32_t f = 0; f < n_faces; ++f) {
        fcell[2 * (size_t)f] = owner[f];
        int32_t other = -1;
        if (f < n_internal) other = neighbour[f];
        else if (f_fid[f] == f && patch_kind[fpatch[f]] == ISO_PATCH_CYCLIC) other = f_other[f];
        fcell[2 * (size_t)f + 1] = other;
        if (f >= n_internal) bpatch[f - n_internal] = fpatch[f];
    }
    std::vector<double> ptrans(3 * (size_t)std::max(n_patches, 1), 0.0);
    for (int32_t p = 0; p < 3 * n_patches; ++p) ptrans[p] = patch_translation[p];
    // slots per cell sorted by face id
    int W = 0;
    std::vector<std::vector<std::array<int32_t, 3>>> slots(n_cells);
    for (int32_t c = 0; c < n_cells; ++c) {
        for (int k = 0; k < ncf[c]; ++k) {
            int32_t f = cface(c, k);
            if (f < 0 || f_fid[f] < 0) continue;
            int s; int32_t other;
            if (f < n_internal) { s = owner[f] == c ? 1 : -1; other = owner[f] == c ? neighbour[f] : owner[f]; }
            else { s = f_sign[f]; other = f_other[f]; }
            slots[c].push_back({f_fid[f], s, other});
        }
        std::sort(slots[c].begin(), slots[c].end(), [](const auto &a, const auto &b) { return a[0] < b[0]; });
        W = std::max<int>(W, (int)slots[c].size());
    }
    W = std::max(W, 1);
    // more than six flux faces: the update kernels come in widths 8, 12 and 16; empty slots pad
    if (W > 6) W = W <= 8 ? 8 : (W <= 12 ? 12 : 16);
    m->W = W;
    std::vector<int32_t> slot_face((size_t)W * n_cells, kEmpty), slot_nbr((size_t)W * n_cells, -1);
    for (int32_t c = 0; c < n_cells; ++c)
        for (size_t k = 0; k < slots[c].size(); ++k) {
            slot_face[k * n_cells + c] = pack_face(slots[c][k][0], slots[c][k][1]);
            slot_nbr[k * n_cells + c] = slots[c][k][2];
        }
    // the update's 32-bit slot words (the layout is described with DevMesh::slot_nar): half the
    // bytes of slot_face + slot_nbr on meshes whose internal faces are numbered by owner, each owner
    // below its neighbour, and whose neighbours lie within 32768 cells
    std::vector<uint32_t> slot_nar;
    uint32_t nar_S = 0;
    {
        int64_t n_slots = 0, n_wide = 0;
        if (n_internal > 0) {
            nar_S = (uint32_t)(((uint64_t)n_internal << 28) / (uint64_t)n_cells);
            slot_nar.assign((size_t)W * n_cells, 0xFFFEu);
            for (int32_t c = 0; c < n_cells; ++c)
                for (size_t k = 0; k < slots[c].size(); ++k) {
                    const int32_t fid = slots[c][k][0], o = slots[c][k][2];
                    const bool own_side = slots[c][k][1] > 0;
                    const int64_t dn = (int64_t)o - c;
                    uint32_t wd = 0xFFFFu;
                    if (fid < n_internal && o >= 0 && dn != 0 && dn >= -32768 && dn <= 32768 && own_side == (c < o)) {
                        const uint32_t owner = (uint32_t)std::min(c, o);
                        const int64_t d = (int64_t)fid - (int64_t)(((uint64_t)owner * nar_S) >> 28);
                        if (d >= 0 && d <= 0xFFFD) {
                            const int32_t up = dn > 0 ? (int32_t)dn - 1 : (int32_t)dn;
                            wd = ((uint32_t)(uint16_t)(int16_t)up << 16) | (uint32_t)d;
                        }
                    }
                    slot_nar[k * (size_t)n_cells + c] = wd;
                    ++n_slots;
                    n_wide += wd == 0xFFFFu ? 1 : 0;
                }
        }
        if (n_slots > 0 && n_wide * 10 <= n_slots) m->n_wide_slots = n_wide;
        else slot_nar.clear();
    }
    // the same slots cell-major, (face, neighbour) per slot (DevMesh::slot_pair)
    std::vector<int32_t> slot_pair(2 * (size_t)W * n_cells);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int k = 0; k < W; ++k) {
            slot_pair[2 * ((size_t)c * W + k)] = slot_face[k * (size_t)n_cells + c];
            slot_pair[2 * ((size_t)c * W + k) + 1] = slot_nbr[k * (size_t)n_cells + c];
        }
    std::vector<int32_t> lface(6 * (size_t)n_cells, kEmpty);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int k = 0; k < 6; ++k) {
            int32_t f = lface_actual[6 * (size_t)c + k];
            if (f < 0 || f_fid[f] < 0) continue;
            int s = f < n_internal ? (owner[f] == c ? 1 : -1) : f_sign[f];
            lface[6 * (size_t)c + k] = pack_face(f_fid[f], s);
        }

    // ---- periodic point classes: match the points of paired cyclic faces
    FrameUnion fu(n_points);
    for (int32_t p = 0; p < n_patches; ++p) {
        if (patch_kind[p] != ISO_PATCH_CYCLIC || patch_partner[p] < p) continue;
        int32_t q = patch_partner[p];
        V3 T{patch_translation[3 * p], patch_translation[3 * p + 1], patch_translation[3 * p + 2]};
        for (int32_t i = 0; i < patch_size[p]; ++i) {
            int32_t f = patch_start[p] + i, g = patch_start[q] + i;
            const int32_t *fa = face_pts + face_ptr[f], *gb = face_pts + face_ptr[g];
            const int na = npts(f);
            if (npts(g) != na) {
                iso_mesh_destroy(m);
                return fail(ISO_EMESH, "cyclic face " + std::to_string(f) + " does not match its partner");
            }
            V3 ctr{0, 0, 0};
            for (int a = 0; a < na; ++a) ctr = ctr + P(fa[a]);
            ctr = (1.0 / na) * ctr;
            double h = 0;
            for (int a = 0; a < na; ++a) h = std::max(h, norm(P(fa[a]) - ctr));
            for (int a = 0; a < na; ++a) {
                V3 tgt = P(fa[a]) + T;
                int32_t hit = -1;
                for (int b = 0; b < na; ++b)
                    if (norm(P(gb[b]) - tgt) <= 1e-8 * h) hit = gb[b];
                if (hit < 0) {
                    iso_mesh_destroy(m);
                    return fail(ISO_EMESH, "cyclic face " + std::to_string(f) + " does not match its partner");
                }
                fu.unite(fa[a], hit, T);
            }
        }
    }
    std::vector<int32_t> cls(n_points, -1), root_cls(n_points, -1);
    std::vector<V3> to_root(n_points);
    int32_t n_classes = 0;
    std::vector<int32_t> cls_root;
    for (int32_t p = 0; p < n_points; ++p) {
        int32_t r = fu.find(p, &to_root[p]);
        if (root_cls[r] < 0) { root_cls[r] = n_classes++; cls_root.push_back(r); }
        cls[p] = root_cls[r];
    }
    m->n_classes = n_classes;
    // stencil of each class: every (cell, vertex) whose point is in the class, centre in the root frame
    std::vector<int32_t> cnt(n_classes + 1, 0);
    // the distinct points of cell c (a general polyhedron's from its list)
    auto cell_point = [&](int32_t c, int i) { return cbig[c] >= 0 ? bv_pts[bv_ptr[cbig[c]] + i] : m->cell_pts[8 * (size_t)c + i]; };
    auto cell_npts = [&](int32_t c) { return cbig[c] >= 0 ? bv_ptr[cbig[c] + 1] - bv_ptr[cbig[c]] : m->nvtx[c]; };
    for (int32_t c = 0; c < n_cells; ++c)
        for (int i = 0; i < cell_npts(c); ++i) cnt[cls[cell_point(c, i)] + 1]++;
    for (int32_t k = 0; k < n_classes; ++k) cnt[k + 1] += cnt[k];
    m->st_nnz = cnt[n_classes];
    std::vector<int32_t> st_cell(cnt[n_classes]);
    std::vector<double> st_w(cnt[n_classes]);
    std::vector<int32_t> fillc(n_classes, 0);
    for (int32_t c = 0; c < n_cells; ++c)  // ascending cell id within each stencil
        for (int i = 0; i < cell_npts(c); ++i) {
            int32_t p = cell_point(c, i);
            int32_t k = cls[p];
            int32_t e = cnt[k] + fillc[k]++;
            st_cell[e] = c;
            V3 xc{m->xc[3 * c], m->xc[3 * c + 1], m->xc[3 * c + 2]};
            V3 xr = P(cls_root[k]);
            st_w[e] = 1.0 / norm(xr - (xc + to_root[p]));  // R: inverse centre-to-vertex distance
        }
    for (int32_t k = 0; k < n_classes; ++k) {
        double s = 0;
        for (int32_t e = cnt[k]; e < cnt[k + 1]; ++e) s += st_w[e];
        for (int32_t e = cnt[k]; e < cnt[k + 1]; ++e) st_w[e] /= s;
    }
    // planar faces: the four points within 1e-12 (relative) of their mean plane
    // (bit k: local face k is planar; a triangle always is); bit 8: not a hexahedron; bit 9: not a
    // hexahedron, and every face planar
    std::vector<int32_t> cflags(n_cells, 0);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int k = 0; k < 6; ++k) {
            V3 q[4];
            if (gnp[6 * (size_t)c] != 0) {
                cflags[c] |= 1 << 8;
                const int np = gnp[6 * (size_t)c + k];
                if (np == 3) cflags[c] |= 1 << k;
                if (np != 4) continue;
                for (int i = 0; i < 4; ++i) q[i] = P(m->cell_pts[8 * (size_t)c + gloop[6 * (size_t)c + k][i]]);
            } else {
                for (int i = 0; i < 4; ++i) q[i] = P(m->cell_pts[8 * (size_t)c + kHexFace[k][i]]);
            }
            V3 nrm = cross(q[2] - q[0], q[3] - q[1]);
            double ln = norm(nrm), size = norm(q[2] - q[0]) + norm(q[3] - q[1]);
            V3 mean = 0.25 * (q[0] + q[1] + q[2] + q[3]);
            bool planar = ln > 0;
            for (int i = 0; i < 4 && planar; ++i) planar = std::fabs(dot(q[i] - mean, nrm)) <= 1e-12 * size * ln;
            if (planar) cflags[c] |= 1 << k;
        }
    for (int32_t c = 0; c < n_cells; ++c)  // general polyhedra: bits 8 and 10, nothing per face
        if (cbig[c] >= 0) cflags[c] = (1 << 8) | (1 << 10);
    for (int32_t c = 0; c < n_cells; ++c) {
        if (gnp[6 * (size_t)c] == 0) continue;
        bool all = true;
        for (int k = 0; k < 6; ++k)
            if (gnp[6 * (size_t)c + k] != 0 && !((cflags[c] >> k) & 1)) all = false;
        if (all) cflags[c] |= 1 << 9;
    }
    std::vector<int32_t> cpt(8 * (size_t)n_cells);
    for (size_t i = 0; i < cpt.size(); ++i) cpt[i] = cls[m->cell_pts[i]];
    std::vector<double> cxyz(24 * (size_t)n_cells);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int i = 0; i < 8; ++i) {
            V3 x = P(m->cell_pts[8 * (size_t)c + i]);
            cxyz[24 * (size_t)c + 3 * i] = x.x;
            cxyz[24 * (size_t)c + 3 * i + 1] = x.y;
            cxyz[24 * (size_t)c + 3 * i + 2] = x.z;
        }
    // local face loops of every cell when the mesh has cells other than hexahedra (hexahedra take
    // the canonical loops): bits 3i..3i+2 the local vertex at loop position i, bit 12 a face,
    // bits 16+i whether loop position i runs from the lower to the higher local index
    std::vector<int32_t> cloop;
    if (m->generic) {
        cloop.assign(6 * (size_t)n_cells, 0);
        for (int32_t c = 0; c < n_cells; ++c)
            for (int k = 0; k < 6; ++k) {
                int lv[4];
                if (cbig[c] >= 0) continue;  // taken by the general-polyhedron kernel
                if (gnp[6 * (size_t)c] == 0) {
                    for (int i = 0; i < 4; ++i) lv[i] = kHexFace[k][i];
                } else {
                    if (gnp[6 * (size_t)c + k] == 0) continue;
                    for (int i = 0; i < 4; ++i) lv[i] = gloop[6 * (size_t)c + k][i];
                }
                int32_t word = 1 << 12;
                for (int i = 0; i < 4; ++i) {
                    word |= lv[i] << (3 * i);
                    if (lv[i] < lv[(i + 1) & 3]) word |= 1 << (16 + i);
                }
                cloop[6 * (size_t)c + k] = word;
            }
    }
    // general polyhedra on the device: point classes and coordinates, each face's packed flux face,
    // planarity (every point within 1e-12 of the face size of the mean plane, normal by Newell)
    const bool any_big = bv_ptr.size() > 1;
    int32_t big_face_pts = 0;
    for (size_t k = 0; k + 1 < bl_ptr.size(); ++k) big_face_pts = std::max(big_face_pts, bl_ptr[k + 1] - bl_ptr[k]);
    std::vector<int32_t> bv_cls(bv_pts.size()), bf_face(bf_fid.size(), kEmpty), bf_planar(bf_fid.size(), 0);
    std::vector<double> bv_xyz(3 * bv_pts.size());
    for (size_t i = 0; i < bv_pts.size(); ++i) {
        bv_cls[i] = cls[bv_pts[i]];
        const V3 x = P(bv_pts[i]);
        bv_xyz[3 * i] = x.x; bv_xyz[3 * i + 1] = x.y; bv_xyz[3 * i + 2] = x.z;
    }
    for (int32_t c = 0; c < n_cells; ++c) {
        if (cbig[c] < 0) continue;
        const int b = cbig[c];
        const int32_t *v = &bv_pts[bv_ptr[b]];
        for (int k = bf_ptr[b]; k < bf_ptr[b + 1]; ++k) {
            const int32_t f = bf_fid[k];
            if (f_fid[f] >= 0) {
                const int sg = f < n_internal ? (owner[f] == c ? 1 : -1) : f_sign[f];
                bf_face[k] = pack_face(f_fid[f], sg);
            }
            const int l0 = bl_ptr[k], np = bl_ptr[k + 1] - l0;
            V3 nrm{0, 0, 0}, mean{0, 0, 0};
            double size = 0;
            for (int i = 0; i < np; ++i) {
                const V3 qi = P(v[bl_vtx[l0 + i]]), qj = P(v[bl_vtx[l0 + (i + 1) % np]]);
                nrm = nrm + cross(qi, qj);
                mean = mean + qi;
                size += norm(qj - qi);
            }
            mean = (1.0 / np) * mean;
            const double ln = norm(nrm);
            bool planar = ln > 0;
            for (int i = 0; i < np && planar; ++i)
                planar = std::fabs(dot(P(v[bl_vtx[l0 + i]]) - mean, nrm)) <= 1e-12 * size * ln;
            bf_planar[k] = planar ? 1 : 0;
        }
    }
    m->patch_alpha.assign(std::max(n_patches, 1), 0.0);
    for (int32_t p = 0; p < n_patches; ++p) m->patch_alpha[p] = patch_alpha_in[p];

    // ---- device
    if (hipGetDevice(&m->device) != hipSuccess) { iso_mesh_destroy(m); return fail(ISO_EDEVICE, "no HIP device"); }
    DevMesh &d = m->dev;
    d.n_cells = n_cells; d.n_faces = n_faces; d.n_classes = n_classes; d.W = W; d.n_patches = n_patches;
    d.big_face_pts = big_face_pts;
    d.all_big = all_big ? 1 : 0;
    if (any_big) {
        m->n_big = (int32_t)bv_ptr.size() - 1;
        m->n_bv = (int32_t)bv_pts.size();
        m->n_bf = (int32_t)bf_fid.size();
        m->n_bl = (int32_t)bl_vtx.size();
        // the class of the polyhedron kernel's instantiation that takes this mesh's polyhedra, kept
        // per cell so that an ensemble can give each member's polyhedra their own
        if (big_face_pts > 4)
            for (int32_t c = 0; c < n_cells; ++c)
                if (cbig[c] >= 0) cflags[c] |= 1 << 11;
    }
    d.n_internal = n_internal;
    d.nar_S = nar_S;
    const int32_t *pair_ptr = nullptr;
    iso_status st = ISO_OK;
    if ((st = upload(m, cxyz, &d.cxyz)) || (st = upload(m, cpt, &d.cpt)) || (st = upload(m, m->vol, &d.vol)) ||
        (st = upload(m, slot_face, &d.slot_face)) || (st = upload(m, slot_nbr, &d.slot_nbr)) ||
        (!slot_nar.empty() && (st = upload(m, slot_nar, &d.slot_nar))) ||
        (st = upload(m, slot_pair, &pair_ptr)) ||
        (st = upload(m, lface, &d.lface)) || (st = upload(m, cflags, &d.cflags)) || (st = upload(m, cnt, &d.st_ptr)) || (st = upload(m, st_cell, &d.st_cell)) ||
        (st = upload(m, st_w, &d.st_w)) || (st = upload(m, m->patch_alpha, &d.patch_alpha)) ||
        (st = upload(m, m->xc, &d.ccen)) || (st = upload(m, fcell, &d.fcell)) || (st = upload(m, bpatch, &d.bpatch)) ||
        (st = upload(m, ptrans, &d.ptrans)) || (m->generic && (st = upload(m, cloop, &d.cloop))) ||
        (any_big && ((st = upload(m, cbig, &d.cbig)) || (st = upload(m, bv_ptr, &d.bv_ptr)) ||
                     (st = upload(m, bv_cls, &d.bv_cls)) || (st = upload(m, bv_xyz, &d.bv_xyz)) ||
                     (st = upload(m, bf_ptr, &d.bf_ptr)) || (st = upload(m, bf_face, &d.bf_face)) ||
                     (st = upload(m, bf_planar, &d.bf_planar)) || (st = upload(m, bl_ptr, &d.bl_ptr)) ||
                     (st = upload(m, bl_vtx, &d.bl_vtx))))) {
        iso_mesh_destroy(m);
        return st;
    }
    d.slot_pair = reinterpret_cast<const int2 *>(pair_ptr);
    *out = m;
    return ISO_OK;
}

iso_status iso_mesh_info(const iso_mesh *m, int64_t *info) {
    if (!m || !info) return fail(ISO_EINVAL, "null argument");
    info[0] = m->n_cells; info[1] = m->n_points; info[2] = m->n_faces; info[3] = m->n_flux;
    info[4] = m->n_classes; info[5] = m->W; info[6] = m->device_bytes; info[7] = m->n_wide_slots;
    return ISO_OK;
}

iso_status iso_mesh_cell_points(const iso_mesh *m, int32_t *out) {
    if (!m || !out) return fail(ISO_EINVAL, "null argument");
    std::memcpy(out, m->cell_pts.data(), m->cell_pts.size() * sizeof(int32_t));
    return ISO_OK;
}

iso_status iso_mesh_geometry(const iso_mesh *m, double *vol, double *xc) {
    if (!m || !vol) return fail(ISO_EINVAL, "null argument");
    std::memcpy(vol, m->vol.data(), m->vol.size() * sizeof(double));
    if (xc) std::memcpy(xc, m->xc.data(), m->xc.size() * sizeof(double));
    return ISO_OK;
}

void iso_plan_destroy(iso_plan *p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->work.side) {
        (void)hipStreamSynchronize(p->work.side);
        (void)hipStreamDestroy(p->work.side);
    }
    if (p->work.fork) (void)hipEventDestroy(p->work.fork);
    if (p->work.join) (void)hipEventDestroy(p->work.join);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    if (p->run_stream) (void)hipStreamSynchronize(p->run_stream);
    if (p->run_exec) (void)hipGraphExecDestroy(p->run_exec);
    if (p->run_graph) (void)hipGraphDestroy(p->run_graph);
    if (p->run_in) (void)hipEventDestroy(p->run_in);
    if (p->run_out) (void)hipEventDestroy(p->run_out);
    if (p->run_stream) (void)hipStreamDestroy(p->run_stream);
    for (void *a : p->allocations) (void)hipFree(a);
    if (p->rz_cell) (void)hipFree(p->rz_cell);
    if (p->rz_w) (void)hipFree(p->rz_w);
    if (p->host_counters) (void)hipHostFree(p->host_counters);
    if (p->host_red) (void)hipHostFree(p->host_red);
    delete p;
}

iso_status iso_plan_create(const iso_mesh *mesh, const iso_options *opt, void *stream, iso_plan **out) {
    if (!out || !mesh) return fail(ISO_EINVAL, "null argument");
    *out = nullptr;
    iso_plan *p = new iso_plan();
    p->mesh = mesh;
    if (opt) p->opt = *opt; else iso_options_default(&p->opt);
    const iso_options &o = p->opt;
    if (const iso_status so = check_options(o, mesh); so != ISO_OK) {
        delete p;
        return so;
    }
    p->stream = static_cast<hipStream_t>(stream);
    const int32_t nc = mesh->n_cells, nf = mesh->n_faces;
    DevWork &w = p->work;
    w.cap = o.max_surface > 0 ? std::min(o.max_surface, nc) : nc;
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
        p->allocations.push_back(*ptr);
        return hipMemset(*ptr, 0, std::max<size_t>(bytes, 256)) == hipSuccess;
    };
    bool ok = alloc((void **)&w.counters, kCntNum * sizeof(int32_t)) && alloc((void **)&w.surf, sizeof(int32_t) * w.cap) &&
              alloc((void **)&w.dvs, sizeof(double) * nf) && alloc((void **)&w.olist, sizeof(int32_t) * (size_t)nc) &&
              alloc((void **)&w.tlist, sizeof(int32_t) * 2 * (size_t)nc) && alloc((void **)&w.flist, sizeof(int32_t) * 4 * (size_t)nf) &&
              alloc((void **)&w.cmark, sizeof(int32_t) * 2 * (size_t)nc) && alloc((void **)&w.fmark, sizeof(int32_t) * nf) &&
              alloc((void **)&w.delta, sizeof(double) * 3 * (size_t)nf) && alloc((void **)&w.dvcur, sizeof(double) * nf) &&
              alloc((void **)&w.red, sizeof(double) * kRedSize) && alloc((void **)&w.sbnd, sizeof(double) * (size_t)nc) &&
              alloc((void **)&w.sclip, sizeof(double) * (size_t)nc);
    if (!ok || hipHostMalloc((void **)&p->host_counters, kCntNum * sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void **)&p->host_red, 64 * sizeof(double)) != hipSuccess) {
        iso_plan_destroy(p);
        return fail(ISO_ENOMEM, "plan workspace allocation failed");
    }
    if (mesh->dev.cbig && !mesh->dev.all_big && (hipStreamCreateWithFlags(&w.side, hipStreamNonBlocking) != hipSuccess ||
                           hipEventCreateWithFlags(&w.fork, hipEventDisableTiming) != hipSuccess ||
                           hipEventCreateWithFlags(&w.join, hipEventDisableTiming) != hipSuccess)) {
        iso_plan_destroy(p);
        return fail(ISO_EDEVICE, "side stream creation failed");
    }
    if (hipDeviceSynchronize() != hipSuccess) { iso_plan_destroy(p); return fail(ISO_EDEVICE, "device error at plan creation"); }
    *out = p;
    return ISO_OK;
}

iso_status iso_plan_set_stream(iso_plan *p, void *stream) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    p->stream = static_cast<hipStream_t>(stream);
    return ISO_OK;
}


static iso_status check_inputs_host(iso_plan *p, const double *alpha, const double *phi, const double *U, double dt) {
    const iso_mesh *m = p->mesh;
    std::vector<double> a(m->n_cells), f(m->n_faces), u(3 * (size_t)m->n_cells);
    if (hipStreamSynchronize(p->stream) != hipSuccess ||
        hipMemcpy(a.data(), alpha, a.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(f.data(), phi, f.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(u.data(), U, u.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ISO_EDEVICE, "copy for input check failed");
    for (double x : a) if (!std::isfinite(x)) return fail(ISO_EINVAL, "non-finite alpha");
    for (double x : f) if (!std::isfinite(x)) return fail(ISO_EINVAL, "non-finite phi");
    for (double x : u) if (!std::isfinite(x)) return fail(ISO_EINVAL, "non-finite U");
    // Courant number 0.5 dt sum|phi| / V over each cell's flux faces
    std::vector<int32_t> sf((size_t)m->W * m->n_cells);
    if (hipMemcpy(sf.data(), m->dev.slot_face, sf.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ISO_EDEVICE, "copy for input check failed");
    for (int32_t c = 0; c < m->n_cells; ++c) {
        double s = 0;
        for (int k = 0; k < m->W; ++k) {
            int32_t v = sf[(size_t)k * m->n_cells + c];
            if (v == kEmpty) continue;
            s += std::fabs(f[v >= 0 ? v : ~v]);
        }
        double co = 0.5 * dt * s / m->vol[c];
        if (co > p->opt.max_courant)
            return fail(ISO_ECOURANT, "Courant number " + std::to_string(co) + " in cell " + std::to_string(c));
    }
    return ISO_OK;
}

// phi1/U1: the second time level of an outer iteration (both or neither), averaged in the kernels
static iso_status step_impl(iso_plan *p, const double *alpha, const double *phi, const double *U, double dt,
                            double *alpha_new, iso_step_stats *stats, const iso_trace *trace,
                            const double *phi1 = nullptr, const double *U1 = nullptr) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    const iso_mesh *m = p->mesh;
    if (const iso_status sa = check_step_args(m, alpha, phi, U, dt, alpha_new, phi1, U1); sa != ISO_OK) return sa;
    if (p->opt.check_inputs) {  // each level within the limits: so is their average
        iso_status s = check_inputs_host(p, alpha, phi, U, dt);
        if (s == ISO_OK && phi1) s = check_inputs_host(p, alpha, phi1, U1, dt);
        if (s != ISO_OK) return s;
    }
    (void)hipGetLastError();
    const Params prm = step_params(p->opt);
    StepArgs args{alpha, phi, U, alpha_new, dt, nullptr, phi1, U1};
    hipEvent_t *ev = nullptr;
    if (p->timing_used < p->timing_cap) ev = &p->events[5 * (size_t)p->timing_used++];
    hipError_t e = launch_step(m->dev, p->work, prm, args, trace, launch_cfg(p->opt), stats != nullptr, p->stream, ev);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    if (p->work.cap < m->n_cells && !stats) {  // a limited interface-cell list: check it was enough
        e = hipMemcpyAsync(p->host_counters, p->work.counters, kCntNum * sizeof(int32_t), hipMemcpyDeviceToHost,
                           p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("device error: ") + hipGetErrorString(e));
        if (p->host_counters[8 + kCntOverflow] > 0) return fail(ISO_ENOSPACE, "interface cells exceed max_surface");
    }
    if (stats) {
        e = launch_stats(m->dev, p->work, alpha, alpha_new, p->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(p->host_counters, p->work.counters, kCntNum * sizeof(int32_t),
                                                hipMemcpyDeviceToHost, p->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(p->host_red, p->work.red, 64 * sizeof(double), hipMemcpyDeviceToHost,
                                                p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("device error: ") + hipGetErrorString(e));
        const int32_t *hc = p->host_counters + 8;  // counters of the step just finished
        const double *hr = p->host_red;
        std::memset(stats, 0, sizeof(*stats));
        stats->n_surface = hc[kCntSurf];
        stats->n_flat = hc[kCntFlat];
        stats->n_nonconverged = hc[kCntNonconv];
        stats->n_bound_active = hc[kCntActive0];
        stats->max_root_iter = hc[kCntMaxIter];
        stats->vol_before = hr[0];
        stats->vol_after = hr[1];
        stats->alpha_min = hr[2];
        stats->alpha_max = hr[3];
        stats->vol_clipped = hr[4];
        stats->vol_boundary_flux = hr[5];
        if (hc[kCntOverflow] > 0) return fail(ISO_ENOSPACE, "interface cells exceed max_surface");
    }
    return ISO_OK;
}

iso_status iso_advect_step(iso_plan *p, const double *alpha, const double *phi, const double *U, double dt,
                           double *alpha_new, iso_step_stats *stats) {
    return step_impl(p, alpha, phi, U, dt, alpha_new, stats, nullptr);
}

namespace {
constexpr int32_t kMaxRunGraphSteps = 256;  // longer runs are launched step by step

hipError_t enqueue_run(iso_plan *p, double *alpha, const double *phi, int64_t ps, const double *U, int64_t us,
                       double dt, int32_t n_steps) {
    const iso_mesh *m = p->mesh;
    const Params prm = step_params(p->opt);
    const LaunchCfg cfg = launch_cfg(p->opt);
    hipError_t e = hipSuccess;
    for (int32_t n = 0; n < n_steps && e == hipSuccess; ++n) {
        const double *in = (n & 1) ? p->run_tmp : alpha;
        double *out = (n & 1) ? alpha : p->run_tmp;
        StepArgs args{in, phi + (size_t)n * ps, U + (size_t)n * us, out, dt, nullptr, nullptr, nullptr};
        e = launch_step(m->dev, p->work, prm, args, nullptr, cfg, false, p->run_stream, nullptr);
    }
    if (e == hipSuccess && (n_steps & 1)) e = launch_copy_f64(p->run_tmp, alpha, m->n_cells, p->run_stream);
    return e;
}
}  // namespace

iso_status iso_plan_run(iso_plan *p, double *alpha, const double *phi, int64_t phi_stride, const double *U,
                        int64_t U_stride, double dt, int32_t n_steps) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    if (!alpha || !phi || !U) return fail(ISO_EINVAL, "null array");
    if (n_steps < 0) return fail(ISO_EINVAL, "negative step count");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(ISO_EINVAL, "dt must be positive and finite");
    const iso_mesh *m = p->mesh;
    const int64_t N = m->n_cells, F = m->n_faces;
    if ((phi_stride != 0 && phi_stride < F) || (U_stride != 0 && U_stride < 3 * N) || phi_stride < 0 || U_stride < 0)
        return fail(ISO_EINVAL, "field strides must be 0 or at least one step's fields");
    if (p->opt.check_inputs) return fail(ISO_EINVAL, "check_inputs copies the inputs to the host: not on a run");
    if (p->work.cap < N)
        return fail(ISO_EUNSUPPORTED, "a run needs the interface-cell list at full capacity (max_surface 0)");
    if (n_steps == 0) return ISO_OK;
    if (overlaps(alpha, (size_t)N * 8, phi, ((size_t)(n_steps - 1) * phi_stride + F) * 8) ||
        overlaps(alpha, (size_t)N * 8, U, ((size_t)(n_steps - 1) * U_stride + 3 * N) * 8))
        return fail(ISO_EINVAL, "alpha overlaps the fields");
    if (!p->run_stream) {
        if (hipStreamCreateWithFlags(&p->run_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->run_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->run_out, hipEventDisableTiming) != hipSuccess)
            return fail(ISO_EDEVICE, "stream or event creation failed");
    }
    if (!p->run_tmp) {
        void *t = nullptr;
        if (hipMalloc(&t, (size_t)N * sizeof(double)) != hipSuccess) return fail(ISO_ENOMEM, "hipMalloc failed");
        p->allocations.push_back(t);
        p->run_tmp = static_cast<double *>(t);
    }
    (void)hipGetLastError();
    // order after the caller's work on the plan's stream
    hipError_t e = hipEventRecord(p->run_in, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->run_stream, p->run_in, 0);
    if (e != hipSuccess) return fail(ISO_EDEVICE, "stream ordering failed");
    if (n_steps > kMaxRunGraphSteps) {
        e = enqueue_run(p, alpha, phi, phi_stride, U, U_stride, dt, n_steps);
    } else {
        const iso_plan::RunKey &k = p->run_key;
        const bool hit = p->run_have && k.alpha == alpha && k.phi == phi && k.U == U && k.ps == phi_stride &&
                         k.us == U_stride && k.dt == dt && k.steps == n_steps;
        if (!hit) {
            if (p->run_exec) (void)hipGraphExecDestroy(p->run_exec);
            if (p->run_graph) (void)hipGraphDestroy(p->run_graph);
            p->run_exec = nullptr;
            p->run_graph = nullptr;
            p->run_have = false;
            e = hipStreamBeginCapture(p->run_stream, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                const hipError_t el = enqueue_run(p, alpha, phi, phi_stride, U, U_stride, dt, n_steps);
                e = hipStreamEndCapture(p->run_stream, &p->run_graph);
                if (el != hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&p->run_exec, p->run_graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
            p->run_key = iso_plan::RunKey{alpha, phi, U, phi_stride, U_stride, dt, n_steps};
            p->run_have = true;
        }
        e = hipGraphLaunch(p->run_exec, p->run_stream);
    }
    if (e == hipSuccess) e = hipEventRecord(p->run_out, p->run_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->run_out, 0);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("run failed: ") + hipGetErrorString(e));
    return ISO_OK;
}

iso_status iso_advect_step_traced(iso_plan *p, const double *alpha, const double *phi, const double *U, double dt,
                                  double *alpha_new, iso_step_stats *stats, const iso_trace *trace) {
    return step_impl(p, alpha, phi, U, dt, alpha_new, stats, trace);
}

iso_status iso_advect_step_avg(iso_plan *p, const double *alpha, const double *phi0, const double *phi1,
                               const double *U0, const double *U1, double dt, double *alpha_new,
                               iso_step_stats *stats) {
    if (!phi1 || !U1) return fail(ISO_EINVAL, "null array");
    return step_impl(p, alpha, phi0, U0, dt, alpha_new, stats, nullptr, phi1, U1);
}

iso_status iso_gfm_faces(iso_plan *p, const double *alpha, const double *p_d, double rho_heavy, double rho_light,
                         double gx, double gy, double gz, double *lambda, double *jump, double *beta_w,
                         double *ghost_own, double *ghost_nbr) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    if (!alpha || !p_d || !lambda || !jump || !beta_w || !ghost_own || !ghost_nbr) return fail(ISO_EINVAL, "null array");
    if (!(rho_heavy > 0) || !(rho_light > 0) || !std::isfinite(rho_heavy) || !std::isfinite(rho_light))
        return fail(ISO_EINVAL, "densities must be positive and finite");
    if (!std::isfinite(gx) || !std::isfinite(gy) || !std::isfinite(gz)) return fail(ISO_EINVAL, "g must be finite");
    const iso_mesh *m = p->mesh;
    if (!m->dev.fcell) return fail(ISO_EUNSUPPORTED, "the plan's mesh has no face table");
    const size_t nc = (size_t)m->n_cells * 8, nf = (size_t)m->n_faces * 8;
    double *outs[5] = {lambda, jump, beta_w, ghost_own, ghost_nbr};
    for (int i = 0; i < 5; ++i) {
        if (overlaps(outs[i], nf, alpha, nc) || overlaps(outs[i], nf, p_d, nc))
            return fail(ISO_EINVAL, "a ghost-fluid output overlaps an input");
        for (int j = 0; j < i; ++j)
            if (overlaps(outs[i], nf, outs[j], nf)) return fail(ISO_EINVAL, "ghost-fluid outputs overlap");
    }
    (void)hipGetLastError();
    GfmArgs a{};
    a.fcell = m->dev.fcell; a.bpatch = m->dev.bpatch; a.ptrans = m->dev.ptrans; a.ccen = m->dev.ccen;
    a.alpha = alpha; a.p_d = p_d;
    a.lambda = lambda; a.jump = jump; a.beta_w = beta_w; a.ghost_own = ghost_own; a.ghost_nbr = ghost_nbr;
    a.b_heavy = 1.0 / rho_heavy; a.b_light = 1.0 / rho_light; a.drho = rho_heavy - rho_light;
    a.g[0] = gx; a.g[1] = gy; a.g[2] = gz;
    a.n_faces = m->n_faces; a.n_internal = m->n_internal;
    hipError_t e = launch_gfm_faces(a, p->stream);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return ISO_OK;
}

iso_status iso_plan_set_relaxation(iso_plan *p, int32_t n_zones, const iso_relax_zone *zones, int64_t *n_zone_cells) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    if (n_zones < 0 || (n_zones > 0 && !zones)) return fail(ISO_EINVAL, "bad zone list");
    for (int32_t z = 0; z < n_zones; ++z) {
        const double *d = zones[z].direction;
        const double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        bool finite = std::isfinite(zones[z].length);
        for (int k = 0; k < 3; ++k) finite = finite && std::isfinite(zones[z].origin[k]) && std::isfinite(d[k]);
        if (!finite || !(n > 0) || !std::isfinite(n) || !(zones[z].length > 0))
            return fail(ISO_EINVAL, "zone " + std::to_string(z) + ": direction and length must be finite and non-zero");
    }
    // zone coordinate of each cell centre: chi = ((x - origin) . e) / length, e the unit direction;
    // a cell is in a zone iff 0 <= chi <= 1, and in at most one
    const iso_mesh *m = p->mesh;
    std::vector<int32_t> cells;
    std::vector<double> w;
    const double norm = std::exp(1.0) - 1.0;
    for (int32_t c = 0; c < m->n_cells; ++c) {
        int32_t hit = -1;
        double chi = 0;
        for (int32_t z = 0; z < n_zones; ++z) {
            const double *o = zones[z].origin, *d = zones[z].direction;
            const double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double e0 = d[0] / n, e1 = d[1] / n, e2 = d[2] / n;
            const double *x = &m->xc[3 * (size_t)c];
            const double q = ((x[0] - o[0]) * e0 + (x[1] - o[1]) * e1 + (x[2] - o[2]) * e2) / zones[z].length;
            if (q >= 0.0 && q <= 1.0) {
                if (hit >= 0) return fail(ISO_EINVAL, "cell " + std::to_string(c) + " lies in two relaxation zones");
                hit = z;
                chi = q;
            }
        }
        if (hit < 0) continue;
        cells.push_back(c);
        w.push_back(1.0 - (std::exp(std::pow(chi, 3.5)) - 1.0) / norm);
    }
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->rz_cell) (void)hipFree(p->rz_cell);
    if (p->rz_w) (void)hipFree(p->rz_w);
    p->rz_cell = nullptr; p->rz_w = nullptr; p->rz_n = 0;
    if (!cells.empty()) {
        if (hipMalloc((void **)&p->rz_cell, cells.size() * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&p->rz_w, w.size() * sizeof(double)) != hipSuccess)
            return fail(ISO_ENOMEM, "relaxation zone allocation failed");
        if (hipMemcpy(p->rz_cell, cells.data(), cells.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->rz_w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail(ISO_EDEVICE, "relaxation zone upload failed");
        p->rz_n = (int64_t)cells.size();
    }
    if (n_zone_cells) *n_zone_cells = p->rz_n;
    return ISO_OK;
}

iso_status iso_relax_blend(iso_plan *p, double *alpha, const double *alpha_target) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    if (!alpha || !alpha_target) return fail(ISO_EINVAL, "null array");
    const size_t nc = (size_t)p->mesh->n_cells * 8;
    if (overlaps(alpha, nc, alpha_target, nc)) return fail(ISO_EINVAL, "alpha overlaps alpha_target");
    (void)hipGetLastError();
    hipError_t e = launch_relax_blend(p->rz_cell, p->rz_w, p->rz_n, alpha, alpha_target, p->stream);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return ISO_OK;
}

static iso_status adj_alloc(iso_plan *p) {
    if (p->adj_ready) return ISO_OK;
    const iso_mesh *m = p->mesh;
    const size_t nc = m->n_cells, nf = m->n_faces;
    const size_t S = std::max(1, p->opt.n_bound_iter);
    AdjWork &w = p->adj;
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
        p->allocations.push_back(*ptr);
        return hipMemset(*ptr, 0, std::max<size_t>(bytes, 256)) == hipSuccess;
    };
    const bool ok =
        alloc((void **)&w.counters, kAdjNum * 4) && alloc((void **)&w.x, nc * 8) && alloc((void **)&w.xbar, nc * 8) && alloc((void **)&w.pv, nc * 8) &&
        alloc((void **)&w.cflag, nc * 4) && alloc((void **)&w.list, S * nc * 4) && alloc((void **)&w.tlist, S * nc * 4) &&
        alloc((void **)&w.cmark, 2 * nc * 4) &&
        alloc((void **)&w.tape, S * nc * (4 + 2 * (size_t)m->W) * 8) && alloc((void **)&w.tflag, S * nc * 8) &&
        alloc((void **)&w.dvcur, nf * 8) && alloc((void **)&w.touched, nf * 4) && alloc((void **)&w.delta, 3 * nf * 8) &&
        alloc((void **)&w.dVb, nf * 8) && alloc((void **)&w.phib, nf * 8) && alloc((void **)&w.dvcurbar, nf * 8) &&
        alloc((void **)&w.deltabar, nf * 8) && alloc((void **)&w.vbar, nf * 8) &&
        alloc((void **)&w.gbuf, kAdjG * nc * 8) && alloc((void **)&w.pbar, std::max<size_t>(m->n_classes, 1) * 8) &&
        alloc((void **)&w.dlist, 9 * nc * 8) &&
        alloc((void **)&w.dlist_big, 33 * std::max<size_t>(m->n_big, 1) * 8) &&
        alloc((void **)&w.gbig, kAdjGBig * std::max<size_t>(m->n_big, 1) * 8) &&
        alloc((void **)&p->adj_vert, 8 * nc * 8) && alloc((void **)&p->adj_kind, nc * 4) &&
        alloc((void **)&p->adj_iso, nc * 8) && alloc((void **)&p->adj_dV, nf * 8) && alloc((void **)&p->adj_raw, nc * 8) &&
        alloc((void **)&p->adj_new, nc * 8);
    if (!ok) return fail(ISO_ENOMEM, "adjoint workspace allocation failed");
    w.big_cap = m->n_big;
    if (hipDeviceSynchronize() != hipSuccess) return fail(ISO_EDEVICE, "device error at adjoint workspace setup");
    p->adj_ready = true;
    return ISO_OK;
}

iso_status iso_advect_step_adjoint(iso_plan *p, const double *alpha, const double *phi, const double *U, double dt,
                                   const iso_trace *fwd, const double *alpha_new_bar, double *alpha_bar,
                                   double *phi_bar) {
    if (!p) return fail(ISO_EINVAL, "null plan");
    if (!alpha || !phi || !U || !alpha_new_bar || !alpha_bar || !phi_bar) return fail(ISO_EINVAL, "null array");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(ISO_EINVAL, "dt must be positive and finite");
    if (p->opt.n_bound_iter > kAdjMaxSweeps)
        return fail(ISO_EUNSUPPORTED, "the adjoint takes at most " + std::to_string(kAdjMaxSweeps) + " bounding sweeps");
    if (p->opt.us_mode != 0) return fail(ISO_EUNSUPPORTED, "the adjoint takes U_S = U_P (us_mode 0) only");
    if (fwd && (!fwd->vert_alpha || !fwd->kind || !fwd->iso || !fwd->dV || !fwd->alpha_raw))
        return fail(ISO_EINVAL, "forward trace needs vert_alpha, kind, iso, dV and alpha_raw");
    const iso_mesh *m = p->mesh;
    const size_t nc = (size_t)m->n_cells * 8, nf = (size_t)m->n_faces * 8;
    const void *ins[] = {alpha, phi, U, alpha_new_bar};
    const size_t insz[] = {nc, nf, 3 * nc, nc};
    for (int i = 0; i < 4; ++i)
        if (overlaps(alpha_bar, nc, ins[i], insz[i]) || overlaps(phi_bar, nf, ins[i], insz[i]))
            return fail(ISO_EINVAL, "an adjoint output overlaps an input");
    if (overlaps(alpha_bar, nc, phi_bar, nf)) return fail(ISO_EINVAL, "alpha_bar overlaps phi_bar");
    iso_status st = adj_alloc(p);
    if (st != ISO_OK) return st;
    (void)hipGetLastError();
    const Params prm = step_params(p->opt);
    StepArgs args{alpha, phi, U, p->adj_new, dt, nullptr};
    iso_trace tr{};
    if (!fwd) {  // the forward step of these inputs, keeping what the adjoint needs
        tr.vert_alpha = p->adj_vert;
        tr.kind = p->adj_kind;
        tr.iso = p->adj_iso;
        tr.dV = p->adj_dV;
        tr.alpha_raw = p->adj_raw;
        hipError_t e = launch_step(m->dev, p->work, prm, args, &tr, launch_cfg(p->opt), false, p->stream, nullptr);
        if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("forward launch failed: ") + hipGetErrorString(e));
        fwd = &tr;
    }
    AdjInputs in{fwd->vert_alpha, fwd->kind, fwd->iso, fwd->dV, fwd->alpha_raw, alpha_new_bar, alpha_bar, phi_bar};
    hipError_t e = launch_adjoint(m->dev, prm, args, in, p->adj, p->stream);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("adjoint launch failed: ") + hipGetErrorString(e));
    return ISO_OK;
}

iso_status iso_plan_set_timing(iso_plan *p, int32_t max_steps) {
    if (!p || max_steps < 0) return fail(ISO_EINVAL, "bad argument");
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(ISO_EDEVICE, "stream sync failed");
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    p->timing_cap = p->timing_used = 0;
    for (int32_t i = 0; i < 5 * max_steps; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(ISO_EDEVICE, "hipEventCreate failed");
        p->events.push_back(e);
    }
    p->timing_cap = max_steps;
    return ISO_OK;
}

iso_status iso_plan_timing(iso_plan *p, double *kernel_ms, int32_t *n_steps) {
    if (!p || !kernel_ms || !n_steps) return fail(ISO_EINVAL, "null argument");
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(ISO_EDEVICE, "stream sync failed");
    for (int k = 0; k < 4; ++k) kernel_ms[k] = 0.0;
    for (int32_t st = 0; st < p->timing_used; ++st)
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p->events[5 * (size_t)st + k], p->events[5 * (size_t)st + k + 1]) != hipSuccess)
                return fail(ISO_EDEVICE, "hipEventElapsedTime failed");
            kernel_ms[k] += ms;
        }
    *n_steps = p->timing_used;
    p->timing_used = 0;
    return ISO_OK;
}

}  // extern "C"
