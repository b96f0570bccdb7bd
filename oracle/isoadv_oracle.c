/*
 * isoAdvector advection step: plain, slow CPU oracle in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * GPU library.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline load it; the library itself never does.  It shares no code, header,
 * table or constant with the GPU path.
 *
 * What it computes (Vukcevic, Roenby, Gatin & Jasak, "A sharp free surface
 * finite volume method applied to gravity wave flows", Section 3.2):
 *   given alpha_P(t), U_P and the face fluxes phi_f, predict alpha_P(t+dt) by
 *     alpha_P(t+dt) = alpha_P(t) - (1/V_P) sum_f dV_f                (flux-form update)
 *     dV_f ~= phi_f * int_t^{t+dt} alpha_f^+(tau) dtau                 (Eqs. dV, alphaf)
 *   where alpha_f^+ is the submerged area fraction of face f, obtained by
 *   sweeping the upwind cell's isoface across the face (Eqs. tv, x_41,
 *   aplus1, aplus2, intaplus), the isoface being the isosurface of the
 *   vertex-interpolated volume fraction that cuts off exactly alpha_P V_P.
 *
 * Readings of points the paper leaves open (each is restated where it is used):
 *   R1  vertex values: inverse centre-to-vertex distance weights, power 1, over
 *       the cells sharing the point; periodic images translated into the point's frame.
 *   R2  interface cell: eps < alpha_P < 1 - eps.
 *   R3  isovalue: bracket between consecutive vertex values, take the vertex
 *       value itself if the sub-volume jumps across alpha_P there, else
 *       bisection to round-off.
 *   R4  vertex v is wet iff a_v > alpha0; an edge is cut iff exactly one end is
 *       wet; the cut point is computed from the wet end.
 *   R5  wet part of a face = its vertex walk emitting wet vertices and cut points;
 *       isoface edges = the cut-to-cut parts of those walks; sub-volume by the
 *       divergence theorem over fan triangles (apex: R6).
 *   R6  polygons (isoface, wet parts of faces) are fanned about their perimeter
 *       centroid, which keeps the sub-volume continuous when a cut point meets a
 *       vertex; isoface normal from the summed fan area vector (out of the wet
 *       part), centre = area-weighted fan centroid; U_S = U_P.
 *   R7  face triangles: fan about the vertex mean; A_f = sum of triangle areas.
 *   R8  Eq. aplus2 as printed is not continuous; the reading used is
 *       alpha+(tau) = alpha+(t2) + (A234/A) [1 - ((t3 - tau)/(t3 - t2))^2].
 *   R8a Eq. x_41's ratio of projections is taken from the sorted arrival times,
 *       (t2 - t1)/(t3 - t1), equal in exact arithmetic and free of a zero denominator.
 *   R9  Eq. intaplus: polynomial pieces integrated over their overlap with the
 *       step window, time measured from the start of the step, each piece's
 *       polynomial written about its own end point (t1 for the first piece,
 *       t3 for the second) and each difference of cubes factored as
 *       (b - a)(pa^2 + pa pb + pb^2) over the squared piece length, so that
 *       neither nearby arrival times nor a window far from them cancel.
 *       Arrival times that overflow mean the plane is at rest on the scale
 *       of the step (static case of R10).
 *   R10 U_S . n_S < 0: the construction gives the dry fraction; U_S . n_S = 0:
 *       static wet fraction (points with d <= 0 are wet).
 *   R11 non-interface (or flat) upwind cell: dV_f = alpha_upwind phi_f dt;
 *       inflow boundary uses the patch value.
 *   R12 update sums in ascending flux-face id, owner side negative.
 *   R13 bounding: Jacobi redistribution over outflow faces, then chopping.
 *   R14 outer iterations (Crank-Nicolson, end of Section 3.2): the step takes the
 *       time-averaged fields phi = (phi(t) + phi(t+dt))/2 and U = (U(t) + U(t+dt))/2;
 *       the caller forms them, this file sees one phi and one U.
 *   R15 (us_mode 1) U_S by cell-point interpolation to x_S (the paper names no
 *       scheme): point velocities by R1's weights; the cell split into tetrahedra
 *       (cell centre, vertex mean of a face, two consecutive points of that face)
 *       carrying U_P, the mean of the face's point velocities and the point
 *       velocities; the linear interpolant in the tetrahedron with the largest
 *       smallest barycentric coordinate of x_S (the one containing it).  us_mode 0
 *       keeps U_S = U_P (R6).
 *   R16 ghost-fluid faces after advection (Eqs. 12-20): the jump H = p_d^- - p_d^+
 *       at x_Gamma is (rho^+ - rho^-) g . x_Gamma, which Eq. 3 (p_d = p - rho g . x) with
 *       a continuous pressure and Eq. 7 give; Eq. 15 as printed has the opposite sign.
 *       A cell is wet iff alpha > 1/2; lambda (Eq. 13) is measured from the face's owner,
 *       beta_w (Eq. 18) from its heavy cell; the ghost values are the heavy fluid's p_d
 *       extended to the dry cell (Eq. 20) and the light fluid's extended to the wet cell
 *       (the mirror of Eqs. 17-20).
 *   Loops over cells, points and faces whose iterations are independent run on OpenMP threads
 *   (or_set_threads); every sum keeps its serial order, so results do not depend on the thread
 *   count.
 *   R17 relaxation zones (Section 3, the paragraph on wave generation and absorption): the
 *       paper blends alpha explicitly towards a target after the advection step with the
 *       exponential weight of Jacobsen, Fuhrman & Fredsoe (2012), which it cites without
 *       printing: alpha <- w alpha + (1 - w) alpha_target, w(chi) = 1 - (exp(chi^3.5) - 1)/(e - 1),
 *       chi in [0, 1] the cell centre's distance from the zone's inner edge (w = 1, the computed
 *       solution kept) towards its outer edge (w = 0, the target imposed), over the zone's
 *       length.  A zone is a slab: an inner-edge point, a direction and a length.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_WALL 0
#define OR_EMPTY 1
#define OR_INOUT 2
#define OR_CYCLIC 3

typedef struct {
    double eps_surf;   /* R2 threshold, default 1e-8 */
    double flat_tol;   /* max a_v - min a_v below which a cell is treated as bulk, default 1e-12 */
    double bound_tol;  /* excursions beyond this trigger redistribution, default 1e-12 */
    int n_bound_iter;  /* Jacobi sweeps, default 3 */
    int clip;          /* chop to [0,1], default 1 */
    int max_bisect;    /* default 200 */
    int us_mode;       /* 0: U_S = U_P (R6); 1: cell-point interpolation to x_S (R15) */
} or_opts;

typedef struct {
    double *a_pts;     /* [n_points] vertex values (R1) */
    int *kind;         /* [n_cells] 0 bulk, 1 reconstructed interface cell, 2 flat interface cell */
    double *iso;       /* [n_cells] isovalue alpha0 (reconstructed cells) */
    double *rec;       /* [7*n_cells] x_S, n_S, U_S.n_S (reconstructed cells) */
    double *dV;        /* [n_faces] dV per flux face id, owner->neighbour orientation, before bounding */
    double *alpha_raw; /* [n_cells] update before bounding and chopping */
    int *iters;        /* [n_cells] bisection iterations */
} or_trace;

typedef struct {
    int64_t n_surface, n_flat, n_bound_active;
    int32_t max_iter;
    double vol_before, vol_after, vol_boundary, vol_clipped, alpha_min, alpha_max;
} or_stats;

typedef struct {
    int n_points, n_faces, n_internal, n_cells, n_patches;
    double *P;              /* 3*n_points */
    int *fptr, *fpts;       /* face -> points */
    int *owner, *nbr;       /* nbr[f] = -1 on the boundary */
    int *fpatch;            /* patch of boundary face, -1 inside */
    int *pstart, *psize, *pkind, *ppartner;
    double *ptrans, *palpha;
    /* flux faces */
    int *flux_id;           /* per face: flux-face id it contributes to, -1 none */
    int *flux_sign;         /* per face: +1 if phi[flux_id] > 0 leaves this face's owner cell */
    int *flux_other;        /* per face: cell on the far side, -1 boundary */
    /* face geometry */
    double *fapex;          /* 3*nf vertex mean */
    /* cells */
    int *cfptr, *cfaces;    /* cell -> own faces */
    int *cpptr, *cpts;      /* cell -> distinct points */
    double *xc, *V;
    /* flux entries per cell, ascending flux id */
    int *ceptr, *ce_flux, *ce_sign, *ce_face, *ce_other;
    /* periodic point classes */
    int *prep;              /* representative point of each class */
    double *poff;           /* x_p + poff[p] = position in the representative's frame */
    int *stptr, *st_cell;   /* per representative: stencil cells */
    double *st_off;         /* translation of each stencil cell centre into the rep frame */
} or_mesh;

/* ------------------------------------------------------------------ small vectors */
static void v_sub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void v_cross(const double *a, const double *b, double *o) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double v_norm(const double *a) { return sqrt(v_dot(a, a)); }

/* ------------------------------------------------------------------ mesh */
void or_mesh_free(or_mesh *m) {
    if (!m) return;
    void *ptrs[] = {m->P, m->fptr, m->fpts, m->owner, m->nbr, m->fpatch, m->pstart, m->psize, m->pkind,
                    m->ppartner, m->ptrans, m->palpha, m->flux_id, m->flux_sign, m->flux_other, m->fapex,
                    m->cfptr, m->cfaces, m->cpptr, m->cpts, m->xc, m->V, m->ceptr, m->ce_flux, m->ce_sign,
                    m->ce_face, m->ce_other, m->prep, m->poff, m->stptr, m->st_cell, m->st_off};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(m);
}

static void *xmalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* points of face f listed outward for cell c (reversed when c is the neighbour) */
static int face_points_for(const or_mesh *m, int f, int c, int *out) {
    int n = m->fptr[f + 1] - m->fptr[f];
    const int *fp = m->fpts + m->fptr[f];
    if (m->owner[f] == c) {
        for (int i = 0; i < n; ++i) out[i] = fp[i];
    } else {
        for (int i = 0; i < n; ++i) out[i] = fp[n - 1 - i];
    }
    return n;
}

static int cmp_int(const void *a, const void *b) { int x = *(const int *)a, y = *(const int *)b; return (x > y) - (x < y); }

#define OR_MAXFP 64  /* max points per face and per cell handled by the oracle */

or_mesh *or_mesh_create(int n_points, const double *pts, int n_faces, const int *face_ptr, const int *face_pts,
                        const int *owner, int n_internal, const int *neighbour, int n_cells, int n_patches,
                        const int *pstart, const int *psize, const int *pkind, const int *ppartner,
                        const double *ptrans, const double *palpha, char *err, int errlen) {
    or_mesh *m = (or_mesh *)xmalloc(sizeof(or_mesh));
    m->n_points = n_points; m->n_faces = n_faces; m->n_internal = n_internal; m->n_cells = n_cells;
    m->n_patches = n_patches;
    m->P = (double *)xmalloc(sizeof(double) * 3 * n_points);
    memcpy(m->P, pts, sizeof(double) * 3 * n_points);
    m->fptr = (int *)xmalloc(sizeof(int) * (n_faces + 1));
    memcpy(m->fptr, face_ptr, sizeof(int) * (n_faces + 1));
    m->fpts = (int *)xmalloc(sizeof(int) * face_ptr[n_faces]);
    memcpy(m->fpts, face_pts, sizeof(int) * face_ptr[n_faces]);
    m->owner = (int *)xmalloc(sizeof(int) * n_faces);
    memcpy(m->owner, owner, sizeof(int) * n_faces);
    m->nbr = (int *)xmalloc(sizeof(int) * n_faces);
    for (int f = 0; f < n_faces; ++f) m->nbr[f] = f < n_internal ? neighbour[f] : -1;
    m->pstart = (int *)xmalloc(sizeof(int) * n_patches); memcpy(m->pstart, pstart, sizeof(int) * n_patches);
    m->psize = (int *)xmalloc(sizeof(int) * n_patches); memcpy(m->psize, psize, sizeof(int) * n_patches);
    m->pkind = (int *)xmalloc(sizeof(int) * n_patches); memcpy(m->pkind, pkind, sizeof(int) * n_patches);
    m->ppartner = (int *)xmalloc(sizeof(int) * n_patches); memcpy(m->ppartner, ppartner, sizeof(int) * n_patches);
    m->ptrans = (double *)xmalloc(sizeof(double) * 3 * n_patches); memcpy(m->ptrans, ptrans, sizeof(double) * 3 * n_patches);
    m->palpha = (double *)xmalloc(sizeof(double) * n_patches); memcpy(m->palpha, palpha, sizeof(double) * n_patches);

    m->fpatch = (int *)xmalloc(sizeof(int) * n_faces);
    for (int f = 0; f < n_faces; ++f) m->fpatch[f] = -1;
    for (int p = 0; p < n_patches; ++p)
        for (int f = pstart[p]; f < pstart[p] + psize[p]; ++f) m->fpatch[f] = p;
    for (int f = n_internal; f < n_faces; ++f)
        if (m->fpatch[f] < 0) { snprintf(err, errlen, "boundary face %d in no patch", f); or_mesh_free(m); return NULL; }

    /* flux faces: interior faces, cyclic pairs (primary = face of the lower-numbered patch), inflow/outflow faces */
    m->flux_id = (int *)xmalloc(sizeof(int) * n_faces);
    m->flux_sign = (int *)xmalloc(sizeof(int) * n_faces);
    m->flux_other = (int *)xmalloc(sizeof(int) * n_faces);
    for (int f = 0; f < n_faces; ++f) {
        m->flux_id[f] = -1; m->flux_sign[f] = 0; m->flux_other[f] = -1;
        if (f < n_internal) { m->flux_id[f] = f; m->flux_sign[f] = 1; m->flux_other[f] = m->nbr[f]; continue; }
        int p = m->fpatch[f];
        if (m->pkind[p] == OR_INOUT) { m->flux_id[f] = f; m->flux_sign[f] = 1; m->flux_other[f] = -1; }
        else if (m->pkind[p] == OR_CYCLIC) {
            int q = m->ppartner[p];
            if (q < 0 || q >= n_patches || m->psize[q] != m->psize[p]) {
                snprintf(err, errlen, "cyclic patch %d has no matching partner", p); or_mesh_free(m); return NULL;
            }
            int g = m->pstart[q] + (f - m->pstart[p]);
            int primary = p < q ? f : g;
            m->flux_id[f] = primary;
            m->flux_sign[f] = (primary == f) ? 1 : -1;
            m->flux_other[f] = m->owner[g];
        }
    }

    /* cell -> own faces */
    m->cfptr = (int *)xmalloc(sizeof(int) * (n_cells + 1));
    for (int f = 0; f < n_faces; ++f) {
        m->cfptr[owner[f] + 1]++;
        if (m->nbr[f] >= 0) m->cfptr[m->nbr[f] + 1]++;
    }
    for (int c = 0; c < n_cells; ++c) m->cfptr[c + 1] += m->cfptr[c];
    m->cfaces = (int *)xmalloc(sizeof(int) * m->cfptr[n_cells]);
    int *fill = (int *)xmalloc(sizeof(int) * n_cells);
    for (int f = 0; f < n_faces; ++f) {
        m->cfaces[m->cfptr[owner[f]] + fill[owner[f]]++] = f;
        if (m->nbr[f] >= 0) m->cfaces[m->cfptr[m->nbr[f]] + fill[m->nbr[f]]++] = f;
    }
    free(fill);

    /* cell -> distinct points */
    m->cpptr = (int *)xmalloc(sizeof(int) * (n_cells + 1));
    int *tmp = (int *)xmalloc(sizeof(int) * OR_MAXFP * 8);
    int total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        total = 0;
        for (int c = 0; c < n_cells; ++c) {
            int n = 0;
            for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
                int f = m->cfaces[k];
                for (int i = m->fptr[f]; i < m->fptr[f + 1]; ++i) tmp[n++] = m->fpts[i];
            }
            qsort(tmp, n, sizeof(int), cmp_int);
            int u = 0;
            for (int i = 0; i < n; ++i) if (i == 0 || tmp[i] != tmp[i - 1]) tmp[u++] = tmp[i];
            if (pass == 0) m->cpptr[c + 1] = m->cpptr[c] + u;
            else memcpy(m->cpts + m->cpptr[c], tmp, sizeof(int) * u);
            total += u;
        }
        if (pass == 0) m->cpts = (int *)xmalloc(sizeof(int) * total);
    }
    free(tmp);

    /* face apex = vertex mean (R7) */
    m->fapex = (double *)xmalloc(sizeof(double) * 3 * n_faces);
    for (int f = 0; f < n_faces; ++f) {
        double s[3] = {0, 0, 0};
        int n = m->fptr[f + 1] - m->fptr[f];
        for (int i = m->fptr[f]; i < m->fptr[f + 1]; ++i)
            for (int d = 0; d < 3; ++d) s[d] += m->P[3 * m->fpts[i] + d];
        for (int d = 0; d < 3; ++d) m->fapex[3 * f + d] = s[d] / n;
    }

    /* cell centre: volume centroid of pyramids from the vertex mean; volume about that centre */
    m->xc = (double *)xmalloc(sizeof(double) * 3 * n_cells);
    m->V = (double *)xmalloc(sizeof(double) * n_cells);
    int fp[OR_MAXFP];
    for (int c = 0; c < n_cells; ++c) {
        double xr[3] = {0, 0, 0};
        int np_ = m->cpptr[c + 1] - m->cpptr[c];
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i)
            for (int d = 0; d < 3; ++d) xr[d] += m->P[3 * m->cpts[i] + d];
        for (int d = 0; d < 3; ++d) xr[d] /= np_;
        double vol = 0, mom[3] = {0, 0, 0};
        for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
            int f = m->cfaces[k];
            int n = face_points_for(m, f, c, fp);
            const double *ap = m->fapex + 3 * f;
            for (int i = 0; i < n; ++i) {
                const double *p0 = m->P + 3 * fp[i], *p1 = m->P + 3 * fp[(i + 1) % n];
                double e0[3], e1[3], S[3], g[3], r[3];
                v_sub(p0, ap, e0); v_sub(p1, ap, e1); v_cross(e0, e1, S);
                for (int d = 0; d < 3; ++d) { S[d] *= 0.5; g[d] = (ap[d] + p0[d] + p1[d]) / 3.0; }
                v_sub(g, xr, r);
                double vt = v_dot(S, r) / 3.0;
                vol += vt;
                for (int d = 0; d < 3; ++d) mom[d] += vt * (xr[d] + ap[d] + p0[d] + p1[d]) / 4.0;
            }
        }
        if (!(vol > 0)) { snprintf(err, errlen, "cell %d has non-positive volume", c); or_mesh_free(m); return NULL; }
        for (int d = 0; d < 3; ++d) m->xc[3 * c + d] = mom[d] / vol;
        /* volume again, about the centroid, with the same triangles the sub-volume uses */
        double v2 = 0;
        for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
            int f = m->cfaces[k];
            int n = face_points_for(m, f, c, fp);
            double w[3] = {0, 0, 0};
            for (int i = 0; i < n; ++i) for (int d = 0; d < 3; ++d) w[d] += m->P[3 * fp[i] + d];
            for (int d = 0; d < 3; ++d) w[d] /= n;
            for (int i = 0; i < n; ++i) {
                const double *p0 = m->P + 3 * fp[i], *p1 = m->P + 3 * fp[(i + 1) % n];
                double e0[3], e1[3], S[3], g[3], r[3];
                v_sub(p0, w, e0); v_sub(p1, w, e1); v_cross(e0, e1, S);
                for (int d = 0; d < 3; ++d) { S[d] *= 0.5; g[d] = (w[d] + p0[d] + p1[d]) / 3.0; }
                v_sub(g, m->xc + 3 * c, r);
                v2 += v_dot(S, r) / 3.0;
            }
        }
        m->V[c] = v2;
    }

    /* flux entries per cell, sorted by flux id (R12) */
    m->ceptr = (int *)xmalloc(sizeof(int) * (n_cells + 1));
    for (int c = 0; c < n_cells; ++c) {
        int n = 0;
        for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) if (m->flux_id[m->cfaces[k]] >= 0) ++n;
        m->ceptr[c + 1] = m->ceptr[c] + n;
    }
    int ne = m->ceptr[n_cells];
    m->ce_flux = (int *)xmalloc(sizeof(int) * ne); m->ce_sign = (int *)xmalloc(sizeof(int) * ne);
    m->ce_face = (int *)xmalloc(sizeof(int) * ne); m->ce_other = (int *)xmalloc(sizeof(int) * ne);
    for (int c = 0; c < n_cells; ++c) {
        int e = m->ceptr[c];
        for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
            int f = m->cfaces[k];
            if (m->flux_id[f] < 0) continue;
            m->ce_flux[e] = m->flux_id[f];
            m->ce_face[e] = f;
            if (f < n_internal) {
                m->ce_sign[e] = (m->owner[f] == c) ? 1 : -1;
                m->ce_other[e] = (m->owner[f] == c) ? m->nbr[f] : m->owner[f];
            } else {
                m->ce_sign[e] = m->flux_sign[f];
                m->ce_other[e] = m->flux_other[f];
            }
            ++e;
        }
        /* insertion sort by flux id */
        for (int i = m->ceptr[c] + 1; i < m->ceptr[c + 1]; ++i) {
            for (int j = i; j > m->ceptr[c] && m->ce_flux[j - 1] > m->ce_flux[j]; --j) {
                int t;
                t = m->ce_flux[j]; m->ce_flux[j] = m->ce_flux[j - 1]; m->ce_flux[j - 1] = t;
                t = m->ce_sign[j]; m->ce_sign[j] = m->ce_sign[j - 1]; m->ce_sign[j - 1] = t;
                t = m->ce_face[j]; m->ce_face[j] = m->ce_face[j - 1]; m->ce_face[j - 1] = t;
                t = m->ce_other[j]; m->ce_other[j] = m->ce_other[j - 1]; m->ce_other[j - 1] = t;
            }
        }
    }

    /* periodic point classes: breadth-first over matched point pairs of cyclic faces */
    int *adj_ptr = (int *)xmalloc(sizeof(int) * (n_points + 1));
    int n_pairs = 0;
    for (int p = 0; p < n_patches; ++p) {
        if (m->pkind[p] != OR_CYCLIC) continue;
        for (int f = m->pstart[p]; f < m->pstart[p] + m->psize[p]; ++f) n_pairs += m->fptr[f + 1] - m->fptr[f];
    }
    int *pa = (int *)xmalloc(sizeof(int) * (n_pairs + 1)), *pb = (int *)xmalloc(sizeof(int) * (n_pairs + 1));
    double *pt = (double *)xmalloc(sizeof(double) * 3 * (n_pairs + 1));
    int np2 = 0;
    for (int p = 0; p < n_patches; ++p) {
        if (m->pkind[p] != OR_CYCLIC) continue;
        int q = m->ppartner[p];
        const double *T = m->ptrans + 3 * p;
        for (int i = 0; i < m->psize[p]; ++i) {
            int f = m->pstart[p] + i, g = m->pstart[q] + i;
            double h = 0;  /* face size for the matching tolerance */
            for (int a = m->fptr[f]; a < m->fptr[f + 1]; ++a) {
                double e[3]; v_sub(m->P + 3 * m->fpts[a], m->fapex + 3 * f, e);
                double l = v_norm(e); if (l > h) h = l;
            }
            for (int a = m->fptr[f]; a < m->fptr[f + 1]; ++a) {
                int qa = m->fpts[a];
                double tgt[3] = {m->P[3 * qa] + T[0], m->P[3 * qa + 1] + T[1], m->P[3 * qa + 2] + T[2]};
                int found = -1;
                for (int b = m->fptr[g]; b < m->fptr[g + 1]; ++b) {
                    double e[3]; v_sub(m->P + 3 * m->fpts[b], tgt, e);
                    if (v_norm(e) <= 1e-8 * h) { found = m->fpts[b]; break; }
                }
                if (found < 0) {
                    snprintf(err, errlen, "cyclic face %d point %d has no partner", f, qa);
                    free(pa); free(pb); free(pt); free(adj_ptr); or_mesh_free(m); return NULL;
                }
                pa[np2] = qa; pb[np2] = found;
                for (int d = 0; d < 3; ++d) pt[3 * np2 + d] = T[d];
                ++np2;
            }
        }
    }
    /* adjacency (both directions): x_b = x_a + t */
    for (int i = 0; i < np2; ++i) { adj_ptr[pa[i] + 1]++; adj_ptr[pb[i] + 1]++; }
    for (int p = 0; p < n_points; ++p) adj_ptr[p + 1] += adj_ptr[p];
    int *adj = (int *)xmalloc(sizeof(int) * (2 * np2 + 1));
    double *adjt = (double *)xmalloc(sizeof(double) * 3 * (2 * np2 + 1));
    int *afill = (int *)xmalloc(sizeof(int) * n_points);
    for (int i = 0; i < np2; ++i) {
        int k = adj_ptr[pa[i]] + afill[pa[i]]++;
        adj[k] = pb[i]; for (int d = 0; d < 3; ++d) adjt[3 * k + d] = pt[3 * i + d];
        k = adj_ptr[pb[i]] + afill[pb[i]]++;
        adj[k] = pa[i]; for (int d = 0; d < 3; ++d) adjt[3 * k + d] = -pt[3 * i + d];
    }
    free(afill); free(pa); free(pb); free(pt);
    m->prep = (int *)xmalloc(sizeof(int) * n_points);
    m->poff = (double *)xmalloc(sizeof(double) * 3 * n_points);
    for (int p = 0; p < n_points; ++p) m->prep[p] = -1;
    int *queue = (int *)xmalloc(sizeof(int) * n_points);
    for (int p = 0; p < n_points; ++p) {
        if (m->prep[p] >= 0) continue;
        int qh = 0, qt = 0;
        queue[qt++] = p; m->prep[p] = p;
        m->poff[3 * p] = m->poff[3 * p + 1] = m->poff[3 * p + 2] = 0;
        while (qh < qt) {
            int u = queue[qh++];
            for (int k = adj_ptr[u]; k < adj_ptr[u + 1]; ++k) {
                int v = adj[k];
                if (m->prep[v] >= 0) continue;
                m->prep[v] = p;
                for (int d = 0; d < 3; ++d) m->poff[3 * v + d] = m->poff[3 * u + d] - adjt[3 * k + d];
                queue[qt++] = v;
            }
        }
    }
    free(queue); free(adj); free(adjt); free(adj_ptr);

    /* stencil of each representative: every cell touching any member, centre moved into the rep frame */
    int *pc_ptr = (int *)xmalloc(sizeof(int) * (n_points + 1));
    for (int c = 0; c < n_cells; ++c)
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) pc_ptr[m->cpts[i] + 1]++;
    for (int p = 0; p < n_points; ++p) pc_ptr[p + 1] += pc_ptr[p];
    int *pc = (int *)xmalloc(sizeof(int) * (pc_ptr[n_points] + 1));
    int *pfill = (int *)xmalloc(sizeof(int) * n_points);
    for (int c = 0; c < n_cells; ++c)
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) { int p = m->cpts[i]; pc[pc_ptr[p] + pfill[p]++] = c; }
    free(pfill);
    m->stptr = (int *)xmalloc(sizeof(int) * (n_points + 1));
    for (int p = 0; p < n_points; ++p) m->stptr[m->prep[p] + 1] += pc_ptr[p + 1] - pc_ptr[p];
    for (int p = 0; p < n_points; ++p) m->stptr[p + 1] += m->stptr[p];
    m->st_cell = (int *)xmalloc(sizeof(int) * (m->stptr[n_points] + 1));
    m->st_off = (double *)xmalloc(sizeof(double) * 3 * (m->stptr[n_points] + 1));
    int *sfill = (int *)xmalloc(sizeof(int) * n_points);
    for (int p = 0; p < n_points; ++p) {
        int r = m->prep[p];
        for (int k = pc_ptr[p]; k < pc_ptr[p + 1]; ++k) {
            int s = m->stptr[r] + sfill[r]++;
            m->st_cell[s] = pc[k];
            for (int d = 0; d < 3; ++d) m->st_off[3 * s + d] = m->poff[3 * p + d];
        }
    }
    free(sfill); free(pc); free(pc_ptr);
    return m;
}

int or_mesh_n_flux_entries(const or_mesh *m) { return m->ceptr[m->n_cells]; }

void or_mesh_geometry(const or_mesh *m, double *xc, double *V) {
    if (xc) memcpy(xc, m->xc, sizeof(double) * 3 * m->n_cells);
    if (V) memcpy(V, m->V, sizeof(double) * m->n_cells);
}

/* ------------------------------------------------------------------ R1 vertex values */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }

void or_point_values(const or_mesh *m, const double *alpha, double *a_pts) {
#pragma omp parallel for schedule(static)
    for (int p = 0; p < m->n_points; ++p) {
        if (m->prep[p] != p) continue;
        const double *xp = m->P + 3 * p;
        double num = 0, den = 0;
        for (int s = m->stptr[p]; s < m->stptr[p + 1]; ++s) {
            int c = m->st_cell[s];
            double xcs[3], e[3];
            for (int d = 0; d < 3; ++d) xcs[d] = m->xc[3 * c + d] + m->st_off[3 * s + d];
            v_sub(xp, xcs, e);
            double w = 1.0 / v_norm(e);
            num += w * alpha[c];
            den += w;
        }
        a_pts[p] = num / den;
    }
#pragma omp parallel for schedule(static)
    for (int p = 0; p < m->n_points; ++p) a_pts[p] = a_pts[m->prep[p]];
}

/* ------------------------------------------------------------------ R4/R5 cutting a cell at an isovalue */
typedef struct {
    double vsub;         /* volume of the wet part */
    double S[3];         /* isoface area vector, out of the wet part */
    double xS[3];        /* isoface centre */
    double Swet[3];      /* sum of the area vectors of the wet parts of the cell faces */
    int n_cut;           /* isoface edges */
} or_cut;

#define OR_MAXCUT 128

static void cut_point(const double *xw, double aw, const double *xd, double ad, double iso, double *out) {
    double lam = (iso - aw) / (ad - aw);
    for (int d = 0; d < 3; ++d) out[d] = xw[d] + lam * (xd[d] - xw[d]);
}

/* accumulate the fan about apex of polygon poly[n] into the volume (about xref) and area vector */
static void fan(const double (*poly)[3], int n, const double *apex, const double *xref, double *vol, double *S) {
    for (int i = 0; i < n; ++i) {
        const double *p0 = poly[i], *p1 = poly[(i + 1) % n];
        double e0[3], e1[3], St[3], g[3], r[3];
        v_sub(p0, apex, e0); v_sub(p1, apex, e1); v_cross(e0, e1, St);
        for (int d = 0; d < 3; ++d) { St[d] *= 0.5; g[d] = (apex[d] + p0[d] + p1[d]) / 3.0; }
        v_sub(g, xref, r);
        *vol += v_dot(St, r) / 3.0;
        if (S) for (int d = 0; d < 3; ++d) S[d] += St[d];
    }
}

/* Fan apex of a polygon given by its boundary edges (a[i] -> b[i]; for a closed loop b[i] = a[i+1]):
 * the length-weighted mean of the edge midpoints (perimeter centroid).  When a cut point reaches a
 * vertex the polygon gains or loses a zero-length edge, which does not move this apex, so the fan
 * surface, the sub-volume and the isoface centre stay continuous in the isovalue (reading R6).
 * If every edge has zero length the mean of the edge start points is used. */
static void perimeter_centroid(double (*a)[3], double (*b)[3], int n, int closed_loop, double *out) {
    double L = 0, acc[3] = {0, 0, 0}, mean[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const double *p = a[i], *q = closed_loop ? a[(i + 1) % n] : b[i];
        double e[3];
        v_sub(q, p, e);
        double l = v_norm(e);
        L += l;
        for (int d = 0; d < 3; ++d) { acc[d] += l * 0.5 * (p[d] + q[d]); mean[d] += p[d]; }
    }
    for (int d = 0; d < 3; ++d) out[d] = L > 0 ? acc[d] / L : mean[d] / n;
}

/* tie_wet = 0: vertex wet iff a_v > iso (R4); tie_wet = 1: a_v >= iso, the limit from below at iso */
static int cell_cut(const or_mesh *m, int c, const double *a_pts, double iso, int tie_wet, or_cut *out) {
    const double *xref = m->xc + 3 * c;
    int fp[OR_MAXFP];
    double poly[2 * OR_MAXFP][3];
    double seg_a[OR_MAXCUT][3], seg_b[OR_MAXCUT][3];  /* isoface boundary edges, oriented */
    int nseg = 0;
    double vol = 0;
    double Swet[3] = {0, 0, 0};
    for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
        int f = m->cfaces[k];
        int n = face_points_for(m, f, c, fp);
        int np_ = 0;
        double last_exit[3] = {0, 0, 0};
        int pending = 0, first_is_entry = 0;
        double first_entry[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i) {
            int qi = fp[i], qj = fp[(i + 1) % n];
            double ai = a_pts[qi], aj = a_pts[qj];
            int wi = tie_wet ? ai >= iso : ai > iso, wj = tie_wet ? aj >= iso : aj > iso;
            const double *xi = m->P + 3 * qi, *xj = m->P + 3 * qj;
            if (wi) { for (int d = 0; d < 3; ++d) poly[np_][d] = xi[d]; ++np_; }
            if (wi != wj) {
                double cp[3];
                if (wi) cut_point(xi, ai, xj, aj, iso, cp); else cut_point(xj, aj, xi, ai, iso, cp);
                for (int d = 0; d < 3; ++d) poly[np_][d] = cp[d];
                ++np_;
                if (wi) {  /* leaving the wet part of the face */
                    for (int d = 0; d < 3; ++d) last_exit[d] = cp[d];
                    pending = 1;
                } else {   /* re-entering: the face walk went exit -> entry; the isoface edge runs entry -> exit */
                    if (pending) {
                        if (nseg >= OR_MAXCUT) return -1;
                        for (int d = 0; d < 3; ++d) { seg_a[nseg][d] = cp[d]; seg_b[nseg][d] = last_exit[d]; }
                        ++nseg; pending = 0;
                    } else {
                        first_is_entry = 1;
                        for (int d = 0; d < 3; ++d) first_entry[d] = cp[d];
                    }
                }
            }
        }
        if (pending && first_is_entry) {  /* the walk's last exit pairs with its first entry */
            if (nseg >= OR_MAXCUT) return -1;
            for (int d = 0; d < 3; ++d) { seg_a[nseg][d] = first_entry[d]; seg_b[nseg][d] = last_exit[d]; }
            ++nseg;
        }
        if (np_ >= 3) {
            double apex[3];
            perimeter_centroid(poly, poly, np_, 1, apex);
            fan((const double(*)[3])poly, np_, apex, xref, &vol, Swet);
        }
    }
    out->Swet[0] = Swet[0]; out->Swet[1] = Swet[1]; out->Swet[2] = Swet[2];
    out->S[0] = out->S[1] = out->S[2] = 0;
    out->xS[0] = out->xS[1] = out->xS[2] = 0;
    out->n_cut = nseg;
    if (nseg > 0) {
        double o[3];
        perimeter_centroid(seg_a, seg_b, nseg, 0, o);
        double S[3] = {0, 0, 0};
        for (int s = 0; s < nseg; ++s) {
            double e0[3], e1[3], St[3], g[3], r[3];
            v_sub(seg_a[s], o, e0); v_sub(seg_b[s], o, e1); v_cross(e0, e1, St);
            for (int d = 0; d < 3; ++d) { St[d] *= 0.5; g[d] = (o[d] + seg_a[s][d] + seg_b[s][d]) / 3.0; }
            v_sub(g, xref, r);
            vol += v_dot(St, r) / 3.0;
            for (int d = 0; d < 3; ++d) S[d] += St[d];
        }
        double nrm = v_norm(S);
        for (int d = 0; d < 3; ++d) out->S[d] = S[d];
        if (nrm > 0) {
            double nS[3] = {S[0] / nrm, S[1] / nrm, S[2] / nrm};
            double wsum = 0, xs[3] = {0, 0, 0};
            for (int s = 0; s < nseg; ++s) {
                double e0[3], e1[3], St[3];
                v_sub(seg_a[s], o, e0); v_sub(seg_b[s], o, e1); v_cross(e0, e1, St);
                double w = 0.5 * v_dot(St, nS);
                for (int d = 0; d < 3; ++d) xs[d] += w * (o[d] + seg_a[s][d] + seg_b[s][d]) / 3.0;
                wsum += w;
            }
            for (int d = 0; d < 3; ++d) out->xS[d] = xs[d] / wsum;
        }
    }
    out->vsub = vol;
    return 0;
}

/* ------------------------------------------------------------------ R3 isovalue by bisection */
int or_cell_cut(const or_mesh *m, int c, const double *a_pts, double iso, or_cut *out) {
    return cell_cut(m, c, a_pts, iso, 0, out);
}

static double vol_frac_minus_alpha(const or_mesh *m, int c, const double *a_pts, double iso, int tie_wet, double alpha_c) {
    or_cut cut;
    cell_cut(m, c, a_pts, iso, tie_wet, &cut);
    return cut.vsub / m->V[c] - alpha_c;
}

/* R3 isovalue.  The sub-volume is a smooth (cubic) function of the isovalue between consecutive
 * vertex values and can only jump at a vertex value (the functional form the paper's search
 * exploits).  So: find consecutive distinct vertex values lo < hi with f(lo) > 0 >= f(hi); if the
 * limit of f from below at hi is still positive, f jumps across zero there and the isovalue is hi;
 * otherwise bisect (lo, hi) down to adjacent doubles. */
static double cell_isovalue(const or_mesh *m, int c, const double *a_pts, double alpha_c, int max_iter, int *iters,
                            int *jump) {
    double s[OR_MAXFP * 8] = {0};
    int n = 0;
    for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) s[n++] = a_pts[m->cpts[i]];
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && s[j - 1] > s[j]; --j) { double t = s[j]; s[j] = s[j - 1]; s[j - 1] = t; }
    int u = 0;
    for (int i = 0; i < n; ++i) if (i == 0 || s[i] != s[i - 1]) s[u++] = s[i];
    int it = 0;
    double lo = s[0], hi = s[u - 1], flo = 1.0 - alpha_c;
    for (int j = 1; j < u; ++j) {
        ++it;
        double fj = vol_frac_minus_alpha(m, c, a_pts, s[j], 0, alpha_c);
        if (fj <= 0.0) { lo = s[j - 1]; hi = s[j]; break; }
        flo = fj;
    }
    ++it;
    double fhi = vol_frac_minus_alpha(m, c, a_pts, hi, 1, alpha_c);  /* limit from below at hi */
    if (jump) *jump = fhi > 0.0;
    if (fhi > 0.0) { if (iters) *iters = it; return hi; }
    while (it < max_iter) {
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;  /* bracket is down to adjacent doubles */
        ++it;
        double fm = vol_frac_minus_alpha(m, c, a_pts, mid, 0, alpha_c);
        if (fm == 0.0) { lo = hi = mid; flo = fhi = 0.0; break; }
        if (fm > 0) { lo = mid; flo = fm; } else { hi = mid; fhi = fm; }
    }
    if (iters) *iters = it;
    return fabs(flo) <= fabs(fhi) ? lo : hi;
}

double or_cell_isovalue(const or_mesh *m, int c, const double *a_pts, double alpha_c, int max_iter, int *iters) {
    return cell_isovalue(m, c, a_pts, alpha_c, max_iter, iters, NULL);
}

/* ------------------------------------------------------------------ Eqs. tv, x_41, aplus1/2, intaplus */
/* area of the part of triangle X with (x - xS).n <= 0, divided by the triangle area (R10 static case) */
static double tri_static_fraction(const double X[3][3], const double *xS, const double *nS) {
    double poly[4][3];
    int np_ = 0;
    double d[3];
    for (int k = 0; k < 3; ++k) { double e[3]; v_sub(X[k], xS, e); d[k] = v_dot(e, nS); }
    for (int k = 0; k < 3; ++k) {
        int j = (k + 1) % 3;
        int wk = d[k] <= 0, wj = d[j] <= 0;
        if (wk) { for (int q = 0; q < 3; ++q) poly[np_][q] = X[k][q]; ++np_; }
        if (wk != wj) {
            double lam = d[k] / (d[k] - d[j]);
            for (int q = 0; q < 3; ++q) poly[np_][q] = X[k][q] + lam * (X[j][q] - X[k][q]);
            ++np_;
        }
    }
    double e1[3], e2[3], Sa[3], Sp[3] = {0, 0, 0};
    v_sub(X[1], X[0], e1); v_sub(X[2], X[0], e2); v_cross(e1, e2, Sa);
    double A2 = v_norm(Sa);
    if (!(A2 > 0)) return 0.0;
    for (int i = 1; i + 1 < np_; ++i) {
        double a[3], b[3], s[3];
        v_sub(poly[i], poly[0], a); v_sub(poly[i + 1], poly[0], b); v_cross(a, b, s);
        for (int q = 0; q < 3; ++q) Sp[q] += s[q];
    }
    return v_dot(Sp, Sa) / (A2 * A2);
}

/* Swept fraction F(tau) of a triangle by a plane with arrival times t1<=t2<=t3 (Eq. aplus1 and the
 * reading R8 of Eq. aplus2); the points are already sorted by arrival time. */
typedef struct { double t1, t2, t3, c1, c2; int step; } or_sweep;

static void sweep_setup(const double X[3][3], const double *t, const double *nS, or_sweep *sw) {
    int idx[3] = {0, 1, 2};
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && t[idx[j - 1]] > t[idx[j]]; --j) { int q = idx[j]; idx[j] = idx[j - 1]; idx[j - 1] = q; }
    const double *x1 = X[idx[0]], *x2 = X[idx[1]], *x3 = X[idx[2]];
    sw->t1 = t[idx[0]]; sw->t2 = t[idx[1]]; sw->t3 = t[idx[2]];
    sw->step = !(sw->t3 > sw->t1);
    sw->c1 = sw->c2 = 0;
    if (sw->step) return;
    double x21[3], x31[3], x41[3], x4[3], x43[3], x23[3], cr[3];
    v_sub(x2, x1, x21); v_sub(x3, x1, x31);
    /* Eq. x_41: the ratio of the projections of x_21 and x_31 on the normal is the ratio of the
     * arrival-time differences, which the sort keeps in [0, 1]; projecting the point differences
     * again can round a face nearly parallel to the isoface to a zero denominator */
    double r = (sw->t2 - sw->t1) / (sw->t3 - sw->t1);
    for (int d = 0; d < 3; ++d) { x41[d] = r * x31[d]; x4[d] = x1[d] + x41[d]; }
    v_sub(x4, x3, x43); v_sub(x2, x3, x23);
    v_cross(x31, x21, cr); double A = 0.5 * v_norm(cr);
    if (!(A > 0)) { sw->step = 1; return; }
    v_cross(x41, x21, cr); double A124 = 0.5 * v_norm(cr);
    v_cross(x43, x23, cr); double A234 = 0.5 * v_norm(cr);
    sw->c1 = A124 / A;
    sw->c2 = A234 / A;
}

static double sweep_value(const or_sweep *sw, double tau) {
    if (sw->step) return tau >= sw->t1 ? 1.0 : 0.0;
    if (tau <= sw->t1) return 0.0;
    if (tau >= sw->t3) return 1.0;
    if (tau <= sw->t2) { double q = (tau - sw->t1) / (sw->t2 - sw->t1); return sw->c1 * q * q; }
    double q = (sw->t3 - tau) / (sw->t3 - sw->t2);
    return sw->c1 + sw->c2 * (1.0 - q * q);
}

/* integral of F over [0, dt] (Eq. intaplus with R9) */
static double sweep_integral(const or_sweep *sw, double dt) {
    double I = 0;
    if (sw->step) { double a = sw->t1 > 0 ? sw->t1 : 0; return a < dt ? dt - a : 0.0; }
    if (sw->t2 > sw->t1) {
        double a = sw->t1 > 0 ? sw->t1 : 0, b = sw->t2 < dt ? sw->t2 : dt;
        if (a < b) {
            double h = sw->t2 - sw->t1, ra = (a - sw->t1) / h, rb = (b - sw->t1) / h;
            /* (pb^3 - pa^3)/h^2 = (b - a)(ra^2 + ra rb + rb^2) with ra, rb in [0,1] */
            I += sw->c1 * (b - a) * (ra * ra + ra * rb + rb * rb) / 3.0;
        }
    }
    if (sw->t3 > sw->t2) {
        double a = sw->t2 > 0 ? sw->t2 : 0, b = sw->t3 < dt ? sw->t3 : dt;
        if (a < b) {
            double h = sw->t3 - sw->t2, qa = (sw->t3 - a) / h, qb = (sw->t3 - b) / h;
            I += (sw->c1 + sw->c2) * (b - a) - sw->c2 * (b - a) * (qa * qa + qa * qb + qb * qb) / 3.0;
        }
    }
    { double a = sw->t3 > 0 ? sw->t3 : 0; if (a < dt) I += dt - a; }
    return I;
}

/* wet fraction of a triangle at time tau after the step start (for tests) */
double or_tri_wet_fraction(const double *x9, const double *xS, const double *nS, double un, double tau) {
    double X[3][3];
    for (int k = 0; k < 3; ++k) for (int d = 0; d < 3; ++d) X[k][d] = x9[3 * k + d];
    double t[3];
    int finite = un != 0.0;
    for (int k = 0; k < 3 && finite; ++k) { double e[3]; v_sub(X[k], xS, e); t[k] = v_dot(e, nS) / un; finite = isfinite(t[k]); }  /* Eq. tv */
    if (!finite) return tri_static_fraction((const double(*)[3])X, xS, nS);
    or_sweep sw; sweep_setup((const double(*)[3])X, t, nS, &sw);
    double F = sweep_value(&sw, tau);
    return un > 0 ? F : 1.0 - F;
}

/* time integral over [0, dt] of the wet fraction of a triangle (R9, R10) */
double or_tri_integral(const double *x9, const double *xS, const double *nS, double un, double dt) {
    double X[3][3];
    for (int k = 0; k < 3; ++k) for (int d = 0; d < 3; ++d) X[k][d] = x9[3 * k + d];
    double t[3];
    int finite = un != 0.0;
    for (int k = 0; k < 3 && finite; ++k) { double e[3]; v_sub(X[k], xS, e); t[k] = v_dot(e, nS) / un; finite = isfinite(t[k]); }
    if (!finite) return dt * tri_static_fraction((const double(*)[3])X, xS, nS);
    or_sweep sw; sweep_setup((const double(*)[3])X, t, nS, &sw);
    double I = sweep_integral(&sw, dt);
    return un > 0 ? I : dt - I;
}

/* time-integrated wet fraction of face f seen from cell c: sum_i (A_i/A_f) int alpha_i^+ (R7) */
double or_face_integral(const or_mesh *m, int f, int c, const double *xS, const double *nS, double un, double dt) {
    int fp[OR_MAXFP];
    int n = face_points_for(m, f, c, fp);
    const double *ap = m->fapex + 3 * f;
    double Af = 0, acc = 0;
    for (int i = 0; i < n; ++i) {
        const double *p0 = m->P + 3 * fp[i], *p1 = m->P + 3 * fp[(i + 1) % n];
        double e0[3], e1[3], cr[3];
        v_sub(p0, ap, e0); v_sub(p1, ap, e1); v_cross(e0, e1, cr);
        double Ai = 0.5 * v_norm(cr);
        double x9[9] = {ap[0], ap[1], ap[2], p0[0], p0[1], p0[2], p1[0], p1[1], p1[2]};
        Af += Ai;
        acc += Ai * or_tri_integral(x9, xS, nS, un, dt);
    }
    return acc / Af;
}

/* ------------------------------------------------------------------ the step */
void or_default_opts(or_opts *o) {
    o->eps_surf = 1e-8; o->flat_tol = 1e-12; o->bound_tol = 1e-12;
    o->n_bound_iter = 3; o->clip = 1; o->max_bisect = 200; o->us_mode = 0;
}

/* R15: the velocity at x in cell c by cell-point interpolation.  U_pts holds the point velocities
 * (R1), component-major.  Each face of the cell, fanned about its vertex mean, gives tetrahedra
 * (cell centre, vertex mean, p_i, p_i+1) carrying U_P, the mean of the face's point velocities,
 * U(p_i) and U(p_i+1); the barycentric coordinates of x come from Cramer's rule, and the
 * tetrahedron whose smallest coordinate is largest (the first one met on a tie) gives the value. */
static void cell_point_velocity(const or_mesh *m, int c, const double *U, const double *U_pts, const double *x,
                                double *out) {
    const int nc = m->n_cells, np = m->n_points;
    const double *xc = m->xc + 3 * c;
    const double Up[3] = {U[c], U[nc + c], U[2 * nc + c]};
    double best = -INFINITY;
    for (int d = 0; d < 3; ++d) out[d] = Up[d];
    int fp[OR_MAXFP];
    double r[3];
    v_sub(x, xc, r);
    for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
        int f = m->cfaces[k];
        int n = face_points_for(m, f, c, fp);
        const double *fc = m->fapex + 3 * f;
        double Uf[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) Uf[d] += U_pts[d * np + fp[i]];
        for (int d = 0; d < 3; ++d) Uf[d] /= n;
        for (int i = 0; i < n; ++i) {
            int pa = fp[i], pb = fp[(i + 1) % n];
            double e1[3], e2[3], e3[3], k23[3], kr3[3], k2r[3];
            v_sub(fc, xc, e1);
            v_sub(m->P + 3 * pa, xc, e2);
            v_sub(m->P + 3 * pb, xc, e3);
            v_cross(e2, e3, k23);
            double det = v_dot(e1, k23);
            if (det == 0.0) continue;
            v_cross(r, e3, kr3);
            v_cross(e2, r, k2r);
            double l1 = v_dot(r, k23) / det, l2 = v_dot(e1, kr3) / det, l3 = v_dot(e1, k2r) / det;
            double l0 = 1.0 - l1 - l2 - l3;
            double mn = fmin(fmin(l0, l1), fmin(l2, l3));
            if (mn > best) {
                best = mn;
                for (int d = 0; d < 3; ++d)
                    out[d] = l0 * Up[d] + l1 * Uf[d] + l2 * U_pts[d * np + pa] + l3 * U_pts[d * np + pb];
            }
        }
    }
}

/* Point velocities (R1 weights per component), component-major [3 * n_points]. */
static double *point_velocities(const or_mesh *m, const double *U) {
    const int nc = m->n_cells, np = m->n_points;
    double *U_pts = (double *)xmalloc(sizeof(double) * 3 * np);
    for (int d = 0; d < 3; ++d) or_point_values(m, U + (size_t)d * nc, U_pts + (size_t)d * np);
    return U_pts;
}

/* R15 for one cell and point (tests): computes the point velocities itself. */
void or_cell_point_velocity(const or_mesh *m, int c, const double *U, const double *x, double *out) {
    double *U_pts = point_velocities(m, U);
    cell_point_velocity(m, c, U, U_pts, x, out);
    free(U_pts);
}

static double chop_roundoff(double x, double tol, double V, double *clipped) {
    if (x < 0.0 && x >= -tol) { *clipped += (0.0 - x) * V; return 0.0; }
    if (x > 1.0 && x <= 1.0 + tol) { *clipped += (1.0 - x) * V; return 1.0; }
    return x;
}

int or_step(const or_mesh *m, const or_opts *opt, const double *alpha, const double *phi, const double *U, double dt,
            double *alpha_new, or_trace *tr, or_stats *st) {
    int nc = m->n_cells, nf = m->n_faces;
    double *a_pts = (double *)xmalloc(sizeof(double) * m->n_points);
    int *kind = (int *)xmalloc(sizeof(int) * nc);
    double *rec = (double *)xmalloc(sizeof(double) * 7 * nc);
    double *dV = (double *)xmalloc(sizeof(double) * nf);
    or_stats s;
    memset(&s, 0, sizeof(s));

    /* R1 */
    or_point_values(m, alpha, a_pts);
    double *U_pts = opt->us_mode == 1 ? point_velocities(m, U) : NULL;

    /* R2, R3, R6: interface cells, their isovalue and isoface (kind -1 marks a flat interface
     * cell until the counts are taken) */
    int *its = (int *)xmalloc(sizeof(int) * nc);
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < nc; ++c) {
        kind[c] = 0;
        its[c] = 0;
        double a = alpha[c];
        if (!(a > opt->eps_surf && a < 1.0 - opt->eps_surf)) continue;
        double lo = 1e300, hi = -1e300;
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) {
            double v = a_pts[m->cpts[i]];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        if (!(hi - lo > opt->flat_tol)) { kind[c] = 2; continue; }
        int it = 0;
        double iso = or_cell_isovalue(m, c, a_pts, a, opt->max_bisect, &it);
        its[c] = it;
        or_cut cut;
        or_cell_cut(m, c, a_pts, iso, &cut);
        double nrm = v_norm(cut.S);
        if (!(nrm > 0)) { kind[c] = 2; continue; }
        kind[c] = 1;
        double nS[3] = {cut.S[0] / nrm, cut.S[1] / nrm, cut.S[2] / nrm};
        double Uc[3] = {U[c], U[nc + c], U[2 * nc + c]};  /* U_S = U_P (R6) */
        if (U_pts) cell_point_velocity(m, c, U, U_pts, cut.xS, Uc);  /* R15 */
        double un = v_dot(Uc, nS);
        for (int d = 0; d < 3; ++d) { rec[7 * c + d] = cut.xS[d]; rec[7 * c + 3 + d] = nS[d]; }
        rec[7 * c + 6] = un;
        if (tr && tr->iso) tr->iso[c] = iso;
        if (tr && tr->iters) tr->iters[c] = it;
    }
    for (int c = 0; c < nc; ++c) {
        if (kind[c] != 0) ++s.n_surface;
        if (kind[c] == 2) ++s.n_flat;
        if (its[c] > s.max_iter) s.max_iter = its[c];
    }
    free(its);

    /* Eq. dV, R11: volume transported through each flux face, owner -> neighbour orientation */
#pragma omp parallel for schedule(static)
    for (int f = 0; f < nf; ++f) dV[f] = 0.0;
    /* each face is written by one cell only: its upwind cell, or the owner of an inflow face */
#pragma omp parallel for schedule(dynamic, 256)
    for (int c = 0; c < nc; ++c) {
        for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
            int fid = m->ce_flux[e], sg = m->ce_sign[e];
            double ph = phi[fid];
            double out = sg * ph;  /* outward flux of cell c through this face */
            if (out > 0) {         /* c is the upwind cell */
                if (kind[c] == 1) {
                    double I = or_face_integral(m, m->ce_face[e], c, rec + 7 * c, rec + 7 * c + 3, rec[7 * c + 6], dt);
                    dV[fid] = ph * I;
                } else {
                    dV[fid] = alpha[c] * ph * dt;
                }
            } else if (out < 0 && m->ce_other[e] < 0) {  /* inflow through a boundary face */
                int p = m->fpatch[m->ce_face[e]];
                dV[fid] = m->palpha[p] * ph * dt;
            }
        }
    }
    if (tr && tr->dV) memcpy(tr->dV, dV, sizeof(double) * nf);

    /* flux-form update (R12) */
    double *cur = (double *)xmalloc(sizeof(double) * nc);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        double sum = 0.0;
        for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) sum += m->ce_sign[e] * dV[m->ce_flux[e]];
        cur[c] = alpha[c] - sum / m->V[c];
    }
    for (int c = 0; c < nc; ++c) s.vol_before += alpha[c] * m->V[c];
    if (tr && tr->alpha_raw) memcpy(tr->alpha_raw, cur, sizeof(double) * nc);

    /* R13 bounding: chop round-off excursions, redistribute larger ones over outflow faces (Jacobi), chop */
    double tol = opt->bound_tol;
    /* per-cell clipped volumes of one pass, summed afterwards in cell order */
    double *clipc = (double *)xmalloc(sizeof(double) * nc);
    int *offc = (int *)xmalloc(sizeof(int) * nc);
    if (opt->clip) {
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
            clipc[c] = 0.0;
            cur[c] = chop_roundoff(cur[c], tol, m->V[c], &clipc[c]);
        }
        for (int c = 0; c < nc; ++c) s.vol_clipped += clipc[c];
    }
    double *delta = (double *)xmalloc(sizeof(double) * nf);
    double *dVc = (double *)xmalloc(sizeof(double) * nf);
#pragma omp parallel for schedule(static)
    for (int f = 0; f < nf; ++f) dVc[f] = dV[f];
    for (int it = 0; it < opt->n_bound_iter; ++it) {
#pragma omp parallel for schedule(static)
        for (int f = 0; f < nf; ++f) delta[f] = 0.0;
        int n_off = 0;
        /* each outflow face's correction is written by its upwind cell only */
#pragma omp parallel for schedule(dynamic, 256)
        for (int c = 0; c < nc; ++c) {
            offc[c] = 0;
            double a = cur[c];
            int over = a > 1.0 + tol, under = a < -tol;
            if (!over && !under) continue;
            offc[c] = 1;
            double sumcap = 0.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
                int fid = m->ce_flux[e], sg = m->ce_sign[e];
                double outphi = sg * phi[fid];
                if (!(outphi > 0)) continue;
                double outv = sg * dVc[fid];
                double cap = over ? outphi * dt - outv : outv;
                if (cap > 0) sumcap += cap;
            }
            if (!(sumcap > 0)) continue;
            double need = over ? (a - 1.0) * m->V[c] : -a * m->V[c];
            double r = need / sumcap;
            if (r > 1.0) r = 1.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
                int fid = m->ce_flux[e], sg = m->ce_sign[e];
                double outphi = sg * phi[fid];
                if (!(outphi > 0)) continue;
                double outv = sg * dVc[fid];
                double cap = over ? outphi * dt - outv : outv;
                if (!(cap > 0)) continue;
                double d = cap * r;                 /* change of the outflow of heavy fluid */
                delta[fid] = over ? sg * d : -sg * d;
            }
        }
        for (int c = 0; c < nc; ++c) n_off += offc[c];
        if (it == 0) s.n_bound_active = n_off;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
            double sum = 0.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) sum += m->ce_sign[e] * delta[m->ce_flux[e]];
            cur[c] = cur[c] - sum / m->V[c];
            clipc[c] = 0.0;
            if (opt->clip) cur[c] = chop_roundoff(cur[c], tol, m->V[c], &clipc[c]);
        }
        for (int c = 0; c < nc; ++c) s.vol_clipped += clipc[c];
#pragma omp parallel for schedule(static)
        for (int f = 0; f < nf; ++f) dVc[f] += delta[f];
    }
    if (opt->n_bound_iter == 0) {
        for (int c = 0; c < nc; ++c) if (cur[c] > 1.0 + tol || cur[c] < -tol) ++s.n_bound_active;
    }
    /* volume that left through the boundary, with the redistribution's corrections of boundary
     * faces (the redistribution preserves volume: what it moves out of the domain leaves through
     * an outflow boundary face), so that vol_after = vol_before - vol_boundary + vol_clipped */
    for (int c = 0; c < nc; ++c)
        for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e)
            if (m->ce_other[e] < 0) s.vol_boundary += m->ce_sign[e] * dVc[m->ce_flux[e]];
    if (opt->clip) {
        for (int c = 0; c < nc; ++c) {
            double x = cur[c];
            if (x < 0.0) { s.vol_clipped += (0.0 - x) * m->V[c]; x = 0.0; }
            if (x > 1.0) { s.vol_clipped += (1.0 - x) * m->V[c]; x = 1.0; }
            cur[c] = x;
        }
    }
    s.alpha_min = 1e300; s.alpha_max = -1e300;
    for (int c = 0; c < nc; ++c) {
        alpha_new[c] = cur[c];
        s.vol_after += cur[c] * m->V[c];
        if (cur[c] < s.alpha_min) s.alpha_min = cur[c];
        if (cur[c] > s.alpha_max) s.alpha_max = cur[c];
    }
    if (tr) {
        if (tr->a_pts) memcpy(tr->a_pts, a_pts, sizeof(double) * m->n_points);
        if (tr->kind) memcpy(tr->kind, kind, sizeof(int) * nc);
        if (tr->rec) memcpy(tr->rec, rec, sizeof(double) * 7 * nc);
    }
    if (st) *st = s;
    free(a_pts); free(kind); free(rec); free(dV); free(cur); free(delta); free(dVc); free(U_pts);
    free(clipc); free(offc);
    return 0;
}

/* many steps with steady fields (timing and trajectory tests) */
int or_run(const or_mesh *m, const or_opts *opt, double *alpha, const double *phi, const double *U, double dt, int n_steps) {
    double *tmp = (double *)xmalloc(sizeof(double) * m->n_cells);
    for (int n = 0; n < n_steps; ++n) {
        or_step(m, opt, alpha, phi, U, dt, tmp, NULL, NULL);
        memcpy(alpha, tmp, sizeof(double) * m->n_cells);
    }
    free(tmp);
    return 0;
}

/* isoface of one cell at a given isovalue, for tests: out = vsub, S[3], xS[3], Swet[3], n_cut */
int or_cell_cut_flat(const or_mesh *m, int c, const double *a_pts, double iso, double *out) {
    or_cut cut;
    int r = or_cell_cut(m, c, a_pts, iso, &cut);
    out[0] = cut.vsub;
    for (int d = 0; d < 3; ++d) { out[1 + d] = cut.S[d]; out[4 + d] = cut.xS[d]; out[7 + d] = cut.Swet[d]; }
    out[10] = cut.n_cut;
    return r;
}

/* ------------------------------------------------------------------ R17 relaxation zones
 * zones: 7 numbers per zone, the inner-edge point (3), the direction into the zone (3) and the
 * length.  A cell whose centre projects to chi = ((x - origin) . e) / length in [0, 1] (e the unit
 * direction) is blended; every other cell keeps alpha.  Returns 0, or -1 for a zone with a zero
 * direction or a length that is not positive, or a cell inside two zones. */
static double relax_weight(double chi) { return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / (exp(1.0) - 1.0); }

int or_relax_blend(const or_mesh *m, int n_zones, const double *zones, const double *alpha, const double *target,
                   double *out) {
    for (int z = 0; z < n_zones; ++z) {
        const double *d = zones + 7 * z + 3;
        if (!(v_norm(d) > 0.0) || !(zones[7 * z + 6] > 0.0)) return -1;
    }
    for (int c = 0; c < m->n_cells; ++c) {
        int hit = -1;
        double chi = 0.0;
        for (int z = 0; z < n_zones; ++z) {
            const double *o = zones + 7 * z, *d = zones + 7 * z + 3;
            double n = v_norm(d), e[3] = {d[0] / n, d[1] / n, d[2] / n}, r[3];
            v_sub(m->xc + 3 * c, o, r);
            double q = v_dot(r, e) / zones[7 * z + 6];
            if (q >= 0.0 && q <= 1.0) {
                if (hit >= 0) return -1;
                hit = z; chi = q;
            }
        }
        if (hit < 0) { out[c] = alpha[c]; continue; }
        double w = relax_weight(chi);
        out[c] = w * alpha[c] + (1.0 - w) * target[c];
    }
    return 0;
}

double or_relax_weight(double chi) { return relax_weight(chi); }

/* ------------------------------------------------------------------ R16 ghost-fluid faces
 * For every flux-carrying face with a cell on each side (internal faces and the flux face of a
 * cyclic pair, the far cell's centre translated into the owner's frame), lambda (Eq. 13) when the
 * two cells lie on opposite sides of alpha = 1/2, else -1; the interface point x_Gamma (Eq. 12),
 * the jump H = p_d^- - p_d^+ there (R16), beta_w (Eq. 18, lambda measured from the heavy cell),
 * and the ghost values: ghost_nbr = p_d at the neighbour's centre seen from the owner's fluid,
 * ghost_own = p_d at the owner's centre seen from the neighbour's fluid (Eq. 20 for the heavy
 * fluid's side, its mirror for the light fluid's).  Away from the interface (and on faces with
 * one cell) the ghost values are the plain cell values (p_d of the owner where there is no
 * neighbour), jump and beta_w are 0. */
void or_gfm_faces(const or_mesh *m, const double *alpha, const double *p_d, double rho_heavy, double rho_light,
                  const double *g, double *lambda, double *jump, double *beta_w, double *ghost_own,
                  double *ghost_nbr) {
    const double bp = 1.0 / rho_heavy, bm = 1.0 / rho_light;  /* Eq. 14 */
    for (int f = 0; f < m->n_faces; ++f) {
        int P = m->owner[f];
        lambda[f] = -1.0; jump[f] = 0.0; beta_w[f] = 0.0;
        ghost_own[f] = p_d[P]; ghost_nbr[f] = p_d[P];
        if (m->flux_id[f] != f || m->flux_other[f] < 0) continue;
        int N = m->flux_other[f];
        double xN[3];
        for (int d = 0; d < 3; ++d) xN[d] = m->xc[3 * N + d];
        if (f >= m->n_internal) {  /* cyclic: the far cell's centre in the owner's frame */
            int p = m->fpatch[f];
            for (int d = 0; d < 3; ++d) xN[d] -= m->ptrans[3 * p + d];
        }
        ghost_nbr[f] = p_d[N];
        double aP = alpha[P], aN = alpha[N];
        int wetP = aP > 0.5, wetN = aN > 0.5;
        if (wetP == wetN) continue;
        double lam = (aP - 0.5) / (aP - aN);  /* Eq. 13 */
        double xG[3];
        for (int d = 0; d < 3; ++d) xG[d] = m->xc[3 * P + d] + lam * (xN[d] - m->xc[3 * P + d]);  /* Eq. 12 */
        double H = (rho_heavy - rho_light) * v_dot(g, xG);  /* R16 */
        double lw = wetP ? lam : 1.0 - lam;                  /* distance fraction from the heavy cell */
        double bw = lw * bm + (1.0 - lw) * bp;               /* Eq. 18 */
        double pW = wetP ? p_d[P] : p_d[N], pD = wetP ? p_d[N] : p_d[P];
        double to_dry = (bm / bw) * pD + (1.0 - bm / bw) * pW - (bm / bw) * H;  /* Eq. 20 */
        double to_wet = (bp / bw) * pW + (1.0 - bp / bw) * pD + (bp / bw) * H;  /* its mirror */
        lambda[f] = lam; jump[f] = H; beta_w[f] = bw;
        ghost_nbr[f] = wetP ? to_dry : to_wet;
        ghost_own[f] = wetP ? to_wet : to_dry;
    }
}

/* ==================================================================================================
 * Tangent of the step (directional derivative with respect to alpha and phi), by the complex step.
 *
 * Every quantity that depends on alpha or phi is carried as x + i h x' with h tiny, through the same
 * arithmetic as the step above; branches, comparisons and sorting use the real parts, so the real
 * parts reproduce the step and Im(result)/h is its exact derivative along (x') (no subtraction,
 * hence no cancellation).  Lengths are sqrt(v . v) without conjugation, which keeps every
 * operation analytic.  The isovalue is found on the real parts by the search above; its
 * derivative follows from the volume constraint vsub(iso; a)/V = alpha_P (implicit function):
 * iso' = -(d/dt [vsub(iso; a + t a')/V - alpha_P - t alpha_P'])/(d vsub/d iso / V), both derivatives
 * taken by complex steps.  Where the isovalue sits at a jump of the sub-volume (R3) it is the
 * vertex value itself and moves with it.  Chopped or clipped values are constants.
 * ================================================================================================== */
#include <complex.h>
typedef double complex cplx;

/* h is so small that h^2 underflows to zero: products of two perturbations never reach the real
 * parts, which therefore stay exactly those of the step (a product of a perturbed alpha and a
 * perturbed phi in an empty cell would otherwise leave a real part of order h^2 and flip a chop). */
#define OR_CSTEP 1e-200

static cplx c_dot3(const cplx *a, const cplx *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void c_cross3(const cplx *a, const cplx *b, cplx *o) {
    cplx x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static cplx c_norm3(const cplx *a) { return csqrt(c_dot3(a, a)); }
static void c_sub3(const cplx *a, const cplx *b, cplx *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void c_of(const double *a, cplx *o) { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }

static void cs_point_values(const or_mesh *m, const cplx *alpha, cplx *a_pts) {
    for (int p = 0; p < m->n_points; ++p) {
        if (m->prep[p] != p) continue;
        const double *xp = m->P + 3 * p;
        cplx num = 0;
        double den = 0;
        for (int s = m->stptr[p]; s < m->stptr[p + 1]; ++s) {
            int c = m->st_cell[s];
            double xcs[3], e[3];
            for (int d = 0; d < 3; ++d) xcs[d] = m->xc[3 * c + d] + m->st_off[3 * s + d];
            v_sub(xp, xcs, e);
            double w = 1.0 / v_norm(e);
            num += w * alpha[c];
            den += w;
        }
        a_pts[p] = num / den;
    }
    for (int p = 0; p < m->n_points; ++p) a_pts[p] = a_pts[m->prep[p]];
}

typedef struct {
    cplx vsub, S[3], xS[3];
    int n_cut;
} cs_cut;

static void cs_cut_point(const double *xw, cplx aw, const double *xd, cplx ad, cplx iso, cplx *out) {
    cplx lam = (iso - aw) / (ad - aw);
    for (int d = 0; d < 3; ++d) out[d] = xw[d] + lam * (xd[d] - xw[d]);
}

static void cs_fan(cplx (*poly)[3], int n, const cplx *apex, const double *xref, cplx *vol) {
    for (int i = 0; i < n; ++i) {
        const cplx *p0 = poly[i], *p1 = poly[(i + 1) % n];
        cplx e0[3], e1[3], St[3], r[3];
        c_sub3(p0, apex, e0); c_sub3(p1, apex, e1); c_cross3(e0, e1, St);
        for (int d = 0; d < 3; ++d) { St[d] *= 0.5; r[d] = (apex[d] + p0[d] + p1[d]) / 3.0 - xref[d]; }
        *vol += c_dot3(St, r) / 3.0;
    }
}

static void cs_perimeter_centroid(cplx (*a)[3], cplx (*b)[3], int n, int closed_loop, cplx *out) {
    cplx L = 0, acc[3] = {0, 0, 0}, mean[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const cplx *p = a[i], *q = closed_loop ? a[(i + 1) % n] : b[i];
        cplx e[3];
        c_sub3(q, p, e);
        cplx l = c_norm3(e);
        L += l;
        for (int d = 0; d < 3; ++d) { acc[d] += l * 0.5 * (p[d] + q[d]); mean[d] += p[d]; }
    }
    for (int d = 0; d < 3; ++d) out[d] = creal(L) > 0 ? acc[d] / L : mean[d] / n;
}

/* cell_cut with complex vertex values and isovalue (same walk, same readings R4-R6) */
static int cs_cell_cut(const or_mesh *m, int c, const cplx *a_pts, cplx iso, int tie_wet, cs_cut *out) {
    const double *xref = m->xc + 3 * c;
    int fp[OR_MAXFP];
    cplx poly[2 * OR_MAXFP][3];
    cplx seg_a[OR_MAXCUT][3], seg_b[OR_MAXCUT][3];
    int nseg = 0;
    cplx vol = 0;
    double isor = creal(iso);
    for (int k = m->cfptr[c]; k < m->cfptr[c + 1]; ++k) {
        int f = m->cfaces[k];
        int n = face_points_for(m, f, c, fp);
        int np_ = 0;
        cplx last_exit[3] = {0, 0, 0}, first_entry[3] = {0, 0, 0};
        int pending = 0, first_is_entry = 0;
        for (int i = 0; i < n; ++i) {
            int qi = fp[i], qj = fp[(i + 1) % n];
            cplx ai = a_pts[qi], aj = a_pts[qj];
            int wi = tie_wet ? creal(ai) >= isor : creal(ai) > isor;
            int wj = tie_wet ? creal(aj) >= isor : creal(aj) > isor;
            const double *xi = m->P + 3 * qi, *xj = m->P + 3 * qj;
            if (wi) { c_of(xi, poly[np_]); ++np_; }
            if (wi != wj) {
                cplx cp[3];
                if (wi) cs_cut_point(xi, ai, xj, aj, iso, cp); else cs_cut_point(xj, aj, xi, ai, iso, cp);
                for (int d = 0; d < 3; ++d) poly[np_][d] = cp[d];
                ++np_;
                if (wi) {
                    for (int d = 0; d < 3; ++d) last_exit[d] = cp[d];
                    pending = 1;
                } else if (pending) {
                    if (nseg >= OR_MAXCUT) return -1;
                    for (int d = 0; d < 3; ++d) { seg_a[nseg][d] = cp[d]; seg_b[nseg][d] = last_exit[d]; }
                    ++nseg; pending = 0;
                } else {
                    first_is_entry = 1;
                    for (int d = 0; d < 3; ++d) first_entry[d] = cp[d];
                }
            }
        }
        if (pending && first_is_entry) {
            if (nseg >= OR_MAXCUT) return -1;
            for (int d = 0; d < 3; ++d) { seg_a[nseg][d] = first_entry[d]; seg_b[nseg][d] = last_exit[d]; }
            ++nseg;
        }
        if (np_ >= 3) {
            cplx apex[3];
            cs_perimeter_centroid(poly, poly, np_, 1, apex);
            cs_fan(poly, np_, apex, xref, &vol);
        }
    }
    out->n_cut = nseg;
    for (int d = 0; d < 3; ++d) out->S[d] = out->xS[d] = 0;
    if (nseg > 0) {
        cplx o[3];
        cs_perimeter_centroid(seg_a, seg_b, nseg, 0, o);
        cplx S[3] = {0, 0, 0};
        for (int s = 0; s < nseg; ++s) {
            cplx e0[3], e1[3], St[3], r[3];
            c_sub3(seg_a[s], o, e0); c_sub3(seg_b[s], o, e1); c_cross3(e0, e1, St);
            for (int d = 0; d < 3; ++d) { St[d] *= 0.5; r[d] = (o[d] + seg_a[s][d] + seg_b[s][d]) / 3.0 - xref[d]; }
            vol += c_dot3(St, r) / 3.0;
            for (int d = 0; d < 3; ++d) S[d] += St[d];
        }
        cplx nrm = c_norm3(S);
        for (int d = 0; d < 3; ++d) out->S[d] = S[d];
        if (creal(nrm) > 0) {
            cplx nS[3] = {S[0] / nrm, S[1] / nrm, S[2] / nrm};
            cplx wsum = 0, xs[3] = {0, 0, 0};
            for (int s = 0; s < nseg; ++s) {
                cplx e0[3], e1[3], St[3];
                c_sub3(seg_a[s], o, e0); c_sub3(seg_b[s], o, e1); c_cross3(e0, e1, St);
                cplx w = 0.5 * c_dot3(St, nS);
                for (int d = 0; d < 3; ++d) xs[d] += w * (o[d] + seg_a[s][d] + seg_b[s][d]) / 3.0;
                wsum += w;
            }
            for (int d = 0; d < 3; ++d) out->xS[d] = xs[d] / wsum;
        }
    }
    out->vsub = vol;
    return 0;
}

/* R3 with its derivative: the real isovalue of the real data, then the implicit (or jump) tangent */
static cplx cs_cell_isovalue(const or_mesh *m, int c, const cplx *a_pts, const double *a_re, cplx alpha_c,
                             int max_iter, int *iters) {
    int jump = 0;
    double x = cell_isovalue(m, c, a_re, creal(alpha_c), max_iter, iters, &jump);
    if (jump) {  /* the isovalue is a vertex value and moves with it */
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i)
            if (a_re[m->cpts[i]] == x) return a_pts[m->cpts[i]];
        return x;
    }
    cs_cut cut;
    /* d/dt of G(x; a + t a', alpha + t alpha') at fixed x */
    cs_cell_cut(m, c, a_pts, x, 0, &cut);
    double g_dot = cimag(cut.vsub / m->V[c] - alpha_c) / OR_CSTEP;
    /* dG/dx at the real data */
    cplx *a_r = (cplx *)xmalloc(sizeof(cplx) * m->n_points);
    for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) a_r[m->cpts[i]] = a_re[m->cpts[i]];
    cs_cell_cut(m, c, a_r, x + OR_CSTEP * _Complex_I, 0, &cut);
    free(a_r);
    double g_x = cimag(cut.vsub) / m->V[c] / OR_CSTEP;
    if (!(g_x != 0.0)) return x;
    return x + (-g_dot / g_x) * OR_CSTEP * _Complex_I;
}

/* Time integral over [0, dt] of the wet fraction of a triangle, for the tangent.  The swept
 * fraction of Eqs. aplus1/aplus2 (reading R8) is the area distribution G of the signed distances
 * d_k of the triangle's points from the isoface plane, evaluated at the distance u_n tau the plane
 * has moved (for either sign of u_n; R10); written in the distance, the integral has no division
 * by u_n except at the breakpoints d_k/u_n, which are clamped to the window, so the derivative
 * stays well conditioned when u_n is near zero (where arrival times diverge).  Each piece between
 * breakpoints is a quadratic in tau, integrated exactly (Simpson's rule). */
static cplx cs_area_cdf(int br, cplx z, cplx e1, cplx e2, cplx e3) {
    if (br == 0) return 0.0;
    if (br == 3) return 1.0;
    if (br == 1) return (z - e1) * (z - e1) / ((e3 - e1) * (e2 - e1));
    return 1.0 - (e3 - z) * (e3 - z) / ((e3 - e1) * (e3 - e2));
}

static int cs_area_branch(double z, double e1, double e2, double e3) {
    return z < e1 ? 0 : (z < e2 ? 1 : (z < e3 ? 2 : 3));
}

static cplx cs_tri_integral(const double X[3][3], const cplx *xS, const cplx *nS, cplx un, double dt) {
    cplx d[3];
    for (int k = 0; k < 3; ++k) { cplx xk[3], e[3]; c_of(X[k], xk); c_sub3(xk, xS, e); d[k] = c_dot3(e, nS); }
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && creal(d[j - 1]) > creal(d[j]); --j) { cplx t = d[j]; d[j] = d[j - 1]; d[j - 1] = t; }
    const cplx e1 = d[0], e2 = d[1], e3 = d[2];
    const double r1 = creal(e1), r2 = creal(e2), r3 = creal(e3);
    if (creal(un) == 0.0) {
        int br = cs_area_branch(0.0, r1, r2, r3);
        return dt / 6.0 * (cs_area_cdf(br, 0.0, e1, e2, e3) + 4.0 * cs_area_cdf(br, un * (0.5 * dt), e1, e2, e3) +
                           cs_area_cdf(br, un * dt, e1, e2, e3));
    }
    cplx bk[3] = {e1 / un, e2 / un, e3 / un};
    if (creal(un) < 0.0) { cplx t = bk[0]; bk[0] = bk[2]; bk[2] = t; }  /* increasing time */
    cplx acc = 0.0, a0 = 0.0;
    for (int k = 0; k < 4; ++k) {
        cplx a1 = dt;
        if (k < 3) a1 = creal(bk[k]) <= 0.0 ? 0.0 : (creal(bk[k]) >= dt ? dt : bk[k]);
        if (creal(a1) > creal(a0)) {
            cplx mid = 0.5 * (a0 + a1);
            int br = cs_area_branch(creal(un * mid), r1, r2, r3);
            acc += (a1 - a0) / 6.0 * (cs_area_cdf(br, un * a0, e1, e2, e3) + 4.0 * cs_area_cdf(br, un * mid, e1, e2, e3) +
                                      cs_area_cdf(br, un * a1, e1, e2, e3));
            a0 = a1;
        }
    }
    return acc;
}

static cplx cs_face_integral(const or_mesh *m, int f, int c, const cplx *xS, const cplx *nS, cplx un, double dt) {
    int fp[OR_MAXFP];
    int n = face_points_for(m, f, c, fp);
    const double *ap = m->fapex + 3 * f;
    double Af = 0;
    cplx acc = 0;
    for (int i = 0; i < n; ++i) {
        const double *p0 = m->P + 3 * fp[i], *p1 = m->P + 3 * fp[(i + 1) % n];
        double e0[3], e1[3], cr[3];
        v_sub(p0, ap, e0); v_sub(p1, ap, e1); v_cross(e0, e1, cr);
        double Ai = 0.5 * v_norm(cr);
        double X[3][3];
        for (int d = 0; d < 3; ++d) { X[0][d] = ap[d]; X[1][d] = p0[d]; X[2][d] = p1[d]; }
        Af += Ai;
        acc += Ai * cs_tri_integral((const double(*)[3])X, xS, nS, un, dt);
    }
    return acc / Af;
}

/* A chop or clip that moves a value by at most OR_ROUND only removes round-off (whether such a
 * value lies just inside or just outside a bound is decided by rounding order), so its tangent is
 * kept; a larger one makes the value a constant. */
#define OR_ROUND 1e-14
static cplx cs_to_bound(cplx x, double b) {
    return fabs(creal(x) - b) <= OR_ROUND ? b + cimag(x) * _Complex_I : b;
}

static cplx cs_chop(cplx x, double tol) {
    if (creal(x) < 0.0 && creal(x) >= -tol) return cs_to_bound(x, 0.0);
    if (creal(x) > 1.0 && creal(x) <= 1.0 + tol) return cs_to_bound(x, 1.0);
    return x;
}

/* The step on complex data (same sequence as or_step; clipped values become constants). */
static void cs_step(const or_mesh *m, const or_opts *opt, const cplx *alpha, const cplx *phi, const double *U, double dt,
                    cplx *alpha_new) {
    int nc = m->n_cells, nf = m->n_faces;
    cplx *a_pts = (cplx *)xmalloc(sizeof(cplx) * m->n_points);
    double *a_re = (double *)xmalloc(sizeof(double) * m->n_points);
    int *kind = (int *)xmalloc(sizeof(int) * nc);
    cplx *rec = (cplx *)xmalloc(sizeof(cplx) * 7 * nc);
    cplx *dV = (cplx *)xmalloc(sizeof(cplx) * nf);
    cs_point_values(m, alpha, a_pts);
    for (int p = 0; p < m->n_points; ++p) a_re[p] = creal(a_pts[p]);
    for (int c = 0; c < nc; ++c) {
        kind[c] = 0;
        double a = creal(alpha[c]);
        if (!(a > opt->eps_surf && a < 1.0 - opt->eps_surf)) continue;
        double lo = 1e300, hi = -1e300;
        for (int i = m->cpptr[c]; i < m->cpptr[c + 1]; ++i) {
            double v = a_re[m->cpts[i]];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        if (!(hi - lo > opt->flat_tol)) { kind[c] = 2; continue; }
        int it = 0;
        cplx iso = cs_cell_isovalue(m, c, a_pts, a_re, alpha[c], opt->max_bisect, &it);
        cs_cut cut;
        cs_cell_cut(m, c, a_pts, iso, 0, &cut);
        cplx nrm = c_norm3(cut.S);
        if (!(creal(nrm) > 0)) { kind[c] = 2; continue; }
        kind[c] = 1;
        for (int d = 0; d < 3; ++d) { rec[7 * c + d] = cut.xS[d]; rec[7 * c + 3 + d] = cut.S[d] / nrm; }
        rec[7 * c + 6] = U[c] * rec[7 * c + 3] + U[nc + c] * rec[7 * c + 4] + U[2 * nc + c] * rec[7 * c + 5];
    }
    for (int f = 0; f < nf; ++f) dV[f] = 0.0;
    for (int c = 0; c < nc; ++c)
        for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
            int fid = m->ce_flux[e], sg = m->ce_sign[e];
            cplx ph = phi[fid];
            double out = sg * creal(ph);
            if (out > 0) {
                if (kind[c] == 1)
                    dV[fid] = ph * cs_face_integral(m, m->ce_face[e], c, rec + 7 * c, rec + 7 * c + 3, rec[7 * c + 6], dt);
                else
                    dV[fid] = alpha[c] * ph * dt;
            } else if (out < 0 && m->ce_other[e] < 0) {
                dV[fid] = m->palpha[m->fpatch[m->ce_face[e]]] * ph * dt;
            }
        }
    cplx *cur = (cplx *)xmalloc(sizeof(cplx) * nc);
    for (int c = 0; c < nc; ++c) {
        cplx sum = 0.0;
        for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) sum += m->ce_sign[e] * dV[m->ce_flux[e]];
        cur[c] = alpha[c] - sum / m->V[c];
    }
    double tol = opt->bound_tol;
    if (opt->clip) for (int c = 0; c < nc; ++c) cur[c] = cs_chop(cur[c], tol);
    cplx *delta = (cplx *)xmalloc(sizeof(cplx) * nf);
    cplx *dVc = (cplx *)xmalloc(sizeof(cplx) * nf);
    memcpy(dVc, dV, sizeof(cplx) * nf);
    for (int it = 0; it < opt->n_bound_iter; ++it) {
        for (int f = 0; f < nf; ++f) delta[f] = 0.0;
        for (int c = 0; c < nc; ++c) {
            cplx a = cur[c];
            int over = creal(a) > 1.0 + tol, under = creal(a) < -tol;
            if (!over && !under) continue;
            cplx sumcap = 0.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
                int fid = m->ce_flux[e], sg = m->ce_sign[e];
                cplx outphi = sg * phi[fid];
                if (!(creal(outphi) > 0)) continue;
                cplx outv = sg * dVc[fid];
                cplx cap = over ? outphi * dt - outv : outv;
                if (creal(cap) > 0) sumcap += cap;
            }
            if (!(creal(sumcap) > 0)) continue;
            cplx need = over ? (a - 1.0) * m->V[c] : -a * m->V[c];
            cplx r = need / sumcap;
            if (creal(r) > 1.0) r = 1.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) {
                int fid = m->ce_flux[e], sg = m->ce_sign[e];
                cplx outphi = sg * phi[fid];
                if (!(creal(outphi) > 0)) continue;
                cplx outv = sg * dVc[fid];
                cplx cap = over ? outphi * dt - outv : outv;
                if (!(creal(cap) > 0)) continue;
                cplx d = cap * r;
                delta[fid] = over ? sg * d : -sg * d;
            }
        }
        for (int c = 0; c < nc; ++c) {
            cplx sum = 0.0;
            for (int e = m->ceptr[c]; e < m->ceptr[c + 1]; ++e) sum += m->ce_sign[e] * delta[m->ce_flux[e]];
            cur[c] = cur[c] - sum / m->V[c];
            if (opt->clip) cur[c] = cs_chop(cur[c], tol);
        }
        for (int f = 0; f < nf; ++f) dVc[f] += delta[f];
    }
    if (opt->clip)
        for (int c = 0; c < nc; ++c) {
            if (creal(cur[c]) < 0.0) cur[c] = cs_to_bound(cur[c], 0.0);
            if (creal(cur[c]) > 1.0) cur[c] = cs_to_bound(cur[c], 1.0);
        }
    for (int c = 0; c < nc; ++c) alpha_new[c] = cur[c];
    free(a_pts); free(a_re); free(kind); free(rec); free(dV); free(cur); free(delta); free(dVc);
}

/* alpha_new = step(alpha, phi) and its derivative along (dalpha, dphi): dalpha_new */
int or_step_tlm(const or_mesh *m, const or_opts *opt, const double *alpha, const double *phi, const double *U, double dt,
                const double *dalpha, const double *dphi, double *alpha_new, double *dalpha_new) {
    int nc = m->n_cells, nf = m->n_faces;
    if (opt->us_mode != 0) return -1;  /* the tangent follows U_S = U_P (R6) only */
    cplx *a = (cplx *)xmalloc(sizeof(cplx) * nc);
    cplx *f = (cplx *)xmalloc(sizeof(cplx) * nf);
    cplx *o = (cplx *)xmalloc(sizeof(cplx) * nc);
    for (int c = 0; c < nc; ++c) a[c] = alpha[c] + (dalpha ? dalpha[c] : 0.0) * OR_CSTEP * _Complex_I;
    for (int k = 0; k < nf; ++k) f[k] = phi[k] + (dphi ? dphi[k] : 0.0) * OR_CSTEP * _Complex_I;
    cs_step(m, opt, a, f, U, dt, o);
    for (int c = 0; c < nc; ++c) {
        if (alpha_new) alpha_new[c] = creal(o[c]);
        dalpha_new[c] = cimag(o[c]) / OR_CSTEP;
    }
    free(a); free(f); free(o);
    return 0;
}
