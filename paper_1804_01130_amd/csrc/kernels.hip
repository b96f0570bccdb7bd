// HIP kernels of the isoAdvector step for gfx950 (wave64), FP64.
//
// One step (Section 3.2 of the paper) runs on one stream with no host synchronisation:
//   find_surface   interface cells (eps < alpha < 1-eps), compacted with wave ballots and one
//                  atomic per 4096-cell work-group
//   surface        eight lanes per interface cell: lane v gathers vertex v's value (inverse
//                  distance stencil); lane k < 6 then owns canonical face k.  The group brackets
//                  the isovalue between two consecutive sorted vertex values, then solves the
//                  volume constraint: Newton on the interval's functional form for planar cells
//                  (one isoface edge per lane), Illinois otherwise.  It builds the isoface, and
//                  lane k integrates the submerged fraction of face k over the step when it is an
//                  outflow face (Eqs. tv .. intaplus) -> dV (each face has one upwind cell: no
//                  atomics).  Interface cells that are general polyhedra go to their own
//                  kernel (big.hip), launched on a side stream beside this one
//   update         per cell, gather over its flux faces in ascending face id: dV from the
//                  interface kernel or alpha_upwind*phi*dt; alpha - sum/V; round-off chopping;
//                  cells outside the bounds are listed and compute the first sweep's corrections
//   bound          one kernel per Jacobi sweep: the touched cells apply the sweep's corrections in
//                  face order with chopping, and those still outside the bounds compute the next
//                  sweep's (bounding step at the end of Section 3.2); a one-group kernel leaves
//                  the workspace clean
// Nothing in the step is a dense contraction, so no matrix instructions are used.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"

namespace isoadv {
namespace {

// One face's share of six times the wet sub-volume and of the isoface sums.
struct Part {
    double v6;  // apex . sum of p x q over the face's wet loop
    D3 cseg;    // sum of s0 x s1 over isoface edges on the face
    D3 oacc;    // sum of length x midpoint over those edges
    double oL;  // their total length
};

// Divergence-theorem share of face k for isovalue iso (vertex wet iff a > iso; a >= iso with
// tie_wet, the limit from below).  The wet part of the face is its loop of wet vertices and cut
// points; fanned about any apex q its share is q . sum(p_i x p_i+1), linear in q.  Planar faces
// use a face vertex (the value does not depend on the apex), others the perimeter centroid of the
// wet part.  Isoface edges on the face run from an entry cut back to the preceding exit cut
// (closing the wet part); they are summed for the isoface's own fan, whose apex is the perimeter
// centroid of all isoface edges.
// The loop sum is taken edge by edge: face edge i contributes a x b with a, b its wet end or its
// cut point (nothing when both ends are dry), and each isoface edge, walked from exit to entry,
// closes the loop with the opposite of its own term.  Masked sums are 0/1-weighted (exact for
// finite terms) and the lanes of a wave (different faces, different cells) never diverge.
__device__ __forceinline__ Part face_part(const FaceLane &f, double iso, bool tie_wet) {
    Part r{0.0, {0, 0, 0}, {0, 0, 0}, 0.0};
    bool w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = f.active && (tie_wet ? f.aq[i] >= iso : f.aq[i] > iso);
    D3 cut[4];
    bool exits[4], entries[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        cut[i] = face_cut(f, i, iso, w[i]);
        exits[i] = w[i] && !w[j];
        entries[i] = !w[i] && w[j];
    }
    // isoface edges: each entry pairs with the exit before it, cyclically
    D3 lastexit{0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) lastexit = sel3(exits[i], cut[i], lastexit);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const D3 s0 = cut[i], s1 = lastexit;
        const double m = entries[i] ? 1.0 : 0.0;
        const double l = norm3(s1 - s0);
        r.cseg = r.cseg + m * cross(s0, s1);
        r.oacc = r.oacc + (m * 0.5 * l) * (s0 + s1);
        r.oL += m * l;
        lastexit = sel3(exits[i], cut[i], lastexit);
    }
    // the wet loop's sum: the face edges' terms, and the isoface edges walked exit to entry
    D3 C = r.cseg;
    C = D3{-C.x, -C.y, -C.z};
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        const D3 a = sel3(w[i], f.q[i], cut[i]), b = sel3(w[j], f.q[j], cut[i]);
        C = C + ((w[i] || w[j]) ? 1.0 : 0.0) * cross(a, b);
        cnt += (w[i] ? 1 : 0) + (w[i] != w[j] ? 1 : 0);
    }
    if (cnt >= 3) {
        D3 ap = f.q[0];
        if (!f.planar) {
            // perimeter centroid of the wet loop: its face-edge pieces and its isoface edges
            D3 pacc = r.oacc, psum{0, 0, 0};
            double pl = r.oL;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = (i + 1) & 3;
                const D3 a = sel3(w[i], f.q[i], cut[i]), b = sel3(w[j], f.q[j], cut[i]);
                const double m = (w[i] || w[j]) ? 1.0 : 0.0;
                const double l = norm3(b - a);
                pacc = pacc + (m * 0.5 * l) * (a + b);
                pl += m * l;
                psum = psum + (w[i] ? 1.0 : 0.0) * f.q[i] + (w[i] != w[j] ? 1.0 : 0.0) * cut[i];
            }
            ap = pl > 0.0 ? (1.0 / pl) * pacc : (1.0 / cnt) * psum;
        }
        r.v6 = dot(ap, C);
    }
    return r;
}

// Isoface fan centroid share of face k: sum over its isoface edges of w (o + s0 + s1), and of w,
// with w the fan triangle's area vector (x2) projected on the unit normal n.
__device__ __forceinline__ void face_centre_part(const FaceLane &f, double iso, D3 o, D3 n, D3 &acc, double &ws) {
    acc = D3{0, 0, 0};
    ws = 0.0;
    bool w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = f.active && f.aq[i] > iso;
    D3 cut[4];
    bool exits[4], entries[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        cut[i] = face_cut(f, i, iso, w[i]);
        exits[i] = w[i] && !w[j];
        entries[i] = !w[i] && w[j];
    }
    D3 lastexit{0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) lastexit = sel3(exits[i], cut[i], lastexit);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const D3 s0 = cut[i], s1 = lastexit;
        const double wt = dot(cross(s0 - o, s1 - o), n);
        if (entries[i]) {
            acc = acc + wt * (o + s0 + s1);
            ws += wt;
        }
        lastexit = sel3(exits[i], cut[i], lastexit);
    }
}

// ------------------------------------------------------------------------------------------ interval
// Between two consecutive vertex values the wet/dry pattern w is fixed and every cut point moves
// linearly with the isovalue: p(u) = p0 + u p1, u = iso - xr.  A face's wet-loop sum
// C(u) = sum p_i x p_i+1 and its isoface-edge sum B(u) = sum s0 x s1 are then quadratics in u,
// so on a planar face (apex = a face vertex) its share of six times the sub-volume is
// apex . C(u), a quadratic; the isoface adds o(u) . B(u) with o the perimeter centroid of all
// isoface edges.  With o and do/du from the perimeter sums, the sub-volume and its derivative
// cost one reduction per evaluation, and Newton's method on the bracket finds the isovalue.
struct FaceQuad {
    // the face's isoface edges (at most two on a quadrilateral): entry point s0 + u s1 to exit
    // point e0 + u e1
    D3 s0[2], s1[2], e0[2], e1[2];
    bool on[2];
};

// Cut point on edge i (loop position) at xr and its rate of change with the isovalue.
__device__ __forceinline__ void face_cut_rate(const FaceLane &f, int i, double xr, bool wet_i, D3 &c0, D3 &c1) {
    const int j = (i + 1) & 3;
    c0 = face_cut(f, i, xr, wet_i);
    const bool fwd = (f.fwd >> i) & 1;
    const double dlam = (wet_i == fwd) ? f.inv[i] : -f.inv[i];
    c1 = dlam * (sel3(wet_i, f.q[j], f.q[i]) - sel3(wet_i, f.q[i], f.q[j]));
}

// Coefficients of the face's share for the wet pattern w, about u = iso - xr: the wet loop is
// walked once around the face; each point is p0 + u p1, and every cross product of two
// consecutive points contributes to the u^0, u^1 and u^2 terms of C(u) = sum p_i x p_i+1.
__device__ __forceinline__ void face_quad_share(const FaceLane &f, const bool *w, double xr, double *acoef) {
    const D3 Z{0, 0, 0};
    D3 C0 = Z, C1 = Z, C2 = Z;
    D3 first0 = Z, first1 = Z, prev0 = Z, prev1 = Z;  // first and previous points of the wet loop
    bool have = false;
    int cnt = 0;
    auto emit = [&](bool on, D3 p0, D3 p1) {
        const D3 k0 = cross(prev0, p0), k1 = cross(prev0, p1) + cross(prev1, p0), k2 = cross(prev1, p1);
        const bool link = on && have;
        C0 = sel3(link, C0 + k0, C0);
        C1 = sel3(link, C1 + k1, C1);
        C2 = sel3(link, C2 + k2, C2);
        first0 = sel3(on && !have, p0, first0);
        first1 = sel3(on && !have, p1, first1);
        prev0 = sel3(on, p0, prev0);
        prev1 = sel3(on, p1, prev1);
        have = have || on;
        cnt += on ? 1 : 0;
    };
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        emit(w[i], f.q[i], Z);
        D3 c0, c1;
        face_cut_rate(f, i, xr, w[i], c0, c1);
        emit(w[i] != w[j], c0, c1);
    }
    // close the loop
    C0 = C0 + cross(prev0, first0);
    C1 = C1 + cross(prev0, first1) + cross(prev1, first0);
    C2 = C2 + cross(prev1, first1);
    const bool use = f.active && cnt >= 3;
    acoef[0] = use ? dot(f.q[0], C0) : 0.0;
    acoef[1] = use ? dot(f.q[0], C1) : 0.0;
    acoef[2] = use ? dot(f.q[0], C2) : 0.0;
}

// The face's isoface edges for the wet pattern w (at most two on a quadrilateral): each runs from
// an entry cut back to the preceding exit cut around the face, points p0 + u p1.
__device__ __forceinline__ FaceQuad face_quad_segs(const FaceLane &f, const bool *w, double xr) {
    const D3 Z{0, 0, 0};
    FaceQuad r{{Z, Z}, {Z, Z}, {Z, Z}, {Z, Z}, {false, false}};
    int nsg = 0;
    D3 le0 = Z, le1 = Z, pe0 = Z, pe1 = Z;  // last exit cut; an entry met before any exit
    bool have_le = false, have_pe = false;
    auto seg = [&](bool on, D3 s0, D3 s1, D3 e0, D3 e1) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bool to = on && nsg == k;
            r.s0[k] = sel3(to, s0, r.s0[k]);
            r.s1[k] = sel3(to, s1, r.s1[k]);
            r.e0[k] = sel3(to, e0, r.e0[k]);
            r.e1[k] = sel3(to, e1, r.e1[k]);
            r.on[k] = r.on[k] || to;
        }
        nsg += on ? 1 : 0;
    };
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        const bool exit_ = f.active && w[i] && !w[j], entry = f.active && !w[i] && w[j];
        D3 c0, c1;
        face_cut_rate(f, i, xr, w[i], c0, c1);
        seg(entry && have_le, c0, c1, le0, le1);
        pe0 = sel3(entry && !have_le, c0, pe0);
        pe1 = sel3(entry && !have_le, c1, pe1);
        have_pe = have_pe || (entry && !have_le);
        le0 = sel3(exit_, c0, le0);
        le1 = sel3(exit_, c1, le1);
        have_le = have_le || exit_;
    }
    seg(have_pe, pe0, pe1, le0, le1);
    return r;
}

// One isoface edge of the interval, held by one lane: entry point s0 + u s1 to exit point
// e0 + u e1.  A lane without an edge holds zeros, which contribute exact zeros below.
struct Seg {
    D3 s0, s1, e0, e1;
    bool on;
};

// Per edge at u: its perimeter sums and their rates of change with u, and B(u) = s x e with its
// derivative.
struct Perim {
    D3 oacc, doacc;  // length x midpoint, and its derivative
    double oL, doL;  // length, and its derivative
    D3 Bu, Bd;       // B(u), B'(u)
};

__device__ __forceinline__ Perim seg_eval(const Seg &sg, double u) {
    Perim r;
    const D3 sp = sg.s0 + u * sg.s1, ep = sg.e0 + u * sg.e1;
    const D3 d = ep - sp, dd = sg.e1 - sg.s1;
    const double l = norm3(d);
    const double dl = l > 0.0 ? dot(d, dd) / l : 0.0;
    r.oacc = (0.5 * l) * (sp + ep);
    r.doacc = (0.5 * dl) * (sp + ep) + (0.5 * l) * (sg.s1 + sg.e1);
    r.oL = l;
    r.doL = dl;
    r.Bu = cross(sp, ep);
    r.Bd = cross(sg.s1, ep) + cross(sp, sg.e1);
    return r;
}

// Gives every lane of the group one isoface edge: lane k < 6 keeps the first edge of face k; the
// second edges of saddle faces (all four edges cut) go to lanes 6 and 7, which own no face.
// Returns false when more than two faces of the cell are saddles (the caller then solves with the
// generic sub-volume instead).
__device__ __forceinline__ bool spread_edges(const FaceQuad &fq, int lv, Seg &sg) {
    const uint64_t bal = __ballot(fq.on[1]);
    const uint32_t gm = (uint32_t)(bal >> (__lane_id() & ~(kLanes - 1))) & 0xFFu;
    const uint32_t gm2 = gm & (gm - 1u);
    const int src = lv == 6 ? (gm ? __ffs(gm) - 1 : 0) : (lv == 7 ? (gm2 ? __ffs(gm2) - 1 : 0) : lv);
    const bool take = (lv == 6 && gm != 0u) || (lv == 7 && gm2 != 0u);
    const D3 Z{0, 0, 0};
    auto pull = [&](const D3 &x) { return D3{grp_get(x.x, src), grp_get(x.y, src), grp_get(x.z, src)}; };
    const D3 s0 = pull(fq.s0[1]), s1 = pull(fq.s1[1]), e0 = pull(fq.e0[1]), e1 = pull(fq.e1[1]);
    const bool face = lv < 6;
    sg.s0 = face ? fq.s0[0] : (take ? s0 : Z);
    sg.s1 = face ? fq.s1[0] : (take ? s1 : Z);
    sg.e0 = face ? fq.e0[0] : (take ? e0 : Z);
    sg.e1 = face ? fq.e1[0] : (take ? e1 : Z);
    sg.on = face ? fq.on[0] : take;
    return __popc(gm) <= 2;
}

// Six times the wet sub-volume of the cell (all lanes of the group take part and get the result).
// The isoface's fan apex is the perimeter centroid of its edges; when they all have zero length
// every s0 x s1 is exactly zero, so the apex does not enter and is left at the origin.
__device__ __forceinline__ double cell_vsub6(const FaceLane &f, double iso, bool tie_wet, D3 *o_out, D3 *cseg_out) {
    const Part p = face_part(f, iso, tie_wet);
    const double v6 = grp_sum(p.v6);
    const D3 cseg = grp_sum3(p.cseg), oacc = grp_sum3(p.oacc);
    const double oL = grp_sum(p.oL);
    const D3 o = oL > 0.0 ? (1.0 / oL) * oacc : D3{0, 0, 0};
    if (o_out) *o_out = o;
    if (cseg_out) *cseg_out = cseg;
    return v6 + dot(o, cseg);
}

// ------------------------------------------------------------------------------------------ first guess
__device__ __forceinline__ double pick8(const double (&v)[8], int i) {
    double r = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) r = i == q ? v[q] : r;
    return r;
}

// First guess of the interval (s_k, s_k+1) of the sorted vertex values s that holds the isovalue
// (k in [0, 6], s_k < s_k+1), which orders the probes of the bracket search.  a: the vertex values
// in canonical order.  Hexahedra: the vertex values are taken as a linear field over the cell in its
// own coordinates (0 or 1 along each of its three edge directions, the rate along each the mean
// difference over its four edges), whose volume fraction above x is one minus the distribution
// function of a sum of three uniform variables, in closed form by inclusion and exclusion over the
// eight corners; lane j evaluates it at s_j, and k counts s_1 .. s_6 whose fraction is at least
// alpha_P.  Other cells: the point a fraction 1 - alpha_P of the way from s_0 to s_7.
template <bool kGeneric>
__device__ __forceinline__ int guess_interval(const double (&a)[8], const double (&s)[8], double aP, int lv,
                                              bool hexahedron) {
    bool hit;
    const double x = pick8(s, lv);
    // a hexahedron takes the same guess in either kernel, so that it searches, and ends, alike
    if (!kGeneric || hexahedron) {
        // canonical vertices 0..3 the bottom loop (0 -> 1 along the first direction, 1 -> 2 along the
        // second), 4..7 above them
        double d1 = 0.25 * fabs((a[1] - a[0]) + (a[2] - a[3]) + (a[5] - a[4]) + (a[6] - a[7]));
        double d2 = 0.25 * fabs((a[3] - a[0]) + (a[2] - a[1]) + (a[7] - a[4]) + (a[6] - a[5]));
        double d3 = 0.25 * fabs((a[4] - a[0]) + (a[5] - a[1]) + (a[6] - a[2]) + (a[7] - a[3]));
        double mean = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) mean += a[i];
        const double f0 = 0.125 * mean - 0.5 * (d1 + d2 + d3);  // the fitted field's lowest corner value
        // a rate of zero (data constant along a direction) is lifted to a small fraction of the
        // largest, which keeps the closed form finite and changes the fraction only slightly
        const double dmin = 1e-3 * fmax(d1, fmax(d2, d3));
        d1 = fmax(d1, dmin);
        d2 = fmax(d2, dmin);
        d3 = fmax(d3, dmin);
        double below = 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const double t = fmax(x - (f0 + ((b & 1) ? d1 : 0.0) + ((b & 2) ? d2 : 0.0) + ((b & 4) ? d3 : 0.0)), 0.0);
            const double t3 = t * t * t;
            below += (__popc(b) & 1) ? -t3 : t3;
        }
        hit = below <= (1.0 - aP) * (6.0 * d1 * d2 * d3);
    } else {
        hit = x <= s[0] + (1.0 - aP) * (s[7] - s[0]);
    }
    const uint32_t gm = (uint32_t)(__ballot(hit && lv >= 1 && lv <= 6) >> (__lane_id() & ~(kLanes - 1))) & 0xFFu;
    int k = __popc(gm);
    // an empty interval (tied values): the non-empty one that starts at the tied value, else the
    // one below it
    int up = -1, dn = -1;
#pragma unroll
    for (int q = 6; q >= 0; --q)
        if (q > k && s[q] < s[q + 1]) up = q;
#pragma unroll
    for (int q = 0; q <= 6; ++q)
        if (q < k && s[q] < s[q + 1]) dn = q;
    if (!(pick8(s, k) < pick8(s, k + 1))) k = up >= 0 ? up : dn;
    return k;
}

// ------------------------------------------------------------------------------------------ kernels
constexpr int kFindBlock = 1024, kFindPerThread = 8;
constexpr int kFindWaves = kFindBlock / 64, kFindSlots = kFindPerThread * kFindWaves;  // 128 wave counts
static_assert(kFindSlots == 128, "the block scan gives each lane of one wave two wave counts");

// Interface cells into a list: every thread loads its kFindPerThread cells first (one coalesced
// double per wave and round), each wave counts its hits per round with a ballot, one wave scans
// the block's 128 counts (two per lane) and takes the block's slots with one atomic, and each hit
// lands at its wave's offset plus its rank among the wave's hits.  List order does not affect any
// result.
__global__ void __launch_bounds__(kFindBlock) k_find_surface(const double *__restrict__ alpha, int n, double eps,
                                                             int32_t *__restrict__ list, int32_t cap,
                                                             int32_t *__restrict__ counters,
                                                             int32_t *__restrict__ kind) {
    __shared__ int wcount[kFindSlots];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const size_t base = (size_t)blockIdx.x * kFindBlock * kFindPerThread;
    double a[kFindPerThread];
#pragma unroll
    for (int k = 0; k < kFindPerThread; ++k) {
        const size_t c = base + (size_t)k * kFindBlock + tid;
        a[k] = c < (size_t)n ? alpha[c] : 0.0;
    }
    bool s[kFindPerThread];
    uint64_t mask[kFindPerThread];
#pragma unroll
    for (int k = 0; k < kFindPerThread; ++k) {
        const size_t c = base + (size_t)k * kFindBlock + tid;
        s[k] = c < (size_t)n && interface_cell(a[k], eps);
        if (kind && c < (size_t)n) kind[c] = 0;
        mask[k] = __ballot(s[k]);
        if (lane == 0) wcount[k * kFindWaves + wid] = __popcll(mask[k]);
    }
    __syncthreads();
    if (wid == 0) {
        const int e0 = wcount[2 * lane], e1 = wcount[2 * lane + 1];
        int incl = e0 + e1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        const int total = __shfl(incl, 63, 64);
        int b = 0;
        if (lane == 63 && total > 0) b = atomicAdd(&counters[kCntSurf], total);
        b = __shfl(b, 63, 64);
        const int ex = incl - e0 - e1;
        wcount[2 * lane] = b + ex;
        wcount[2 * lane + 1] = b + ex + e0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFindPerThread; ++k) {
        if (!s[k]) continue;
        const int pos = wcount[k * kFindWaves + wid] +
                        (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask[k] >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mask[k], 0u));
        if (pos < cap) list[pos] = (int32_t)(base + (size_t)k * kFindBlock + tid);
        else atomicAdd(&counters[kCntOverflow], 1);
    }
}

// The flux of face f and the velocity of cell c; with a second time level (outer iterations,
// Crank-Nicolson) their averages, formed as they are read.
template <bool kAvg>
__device__ __forceinline__ double flux_at(const double *phi, const double *phi1, int32_t f) {
    if constexpr (kAvg) return 0.5 * (phi[f] + phi1[f]);
    else return phi[f];
}
__device__ __forceinline__ D3 vel_at(const double *U, const double *U1, int32_t c, size_t n) {
    if (U1) return D3{0.5 * (U[c] + U1[c]), 0.5 * (U[n + c] + U1[n + c]), 0.5 * (U[2 * n + c] + U1[2 * n + c])};
    return D3{U[c], U[n + c], U[2 * n + c]};
}

struct SurfArgs {
    DevMesh m;
    const double *alpha, *phi, *U;
    double dt;
    const double *dt_dom;
    double eps, flat_tol;
    int32_t max_rounds;
    const int32_t *list;
    int32_t *counters;
    int32_t cap;
    double *dvs;
    int want_stats;
    iso_trace tr;
    const double *phi1, *U1;  // second time level, or nullptr
    double root_tol;          // stop the isovalue search at |V_sub/V - alpha| <= root_tol (0: round-off)
};

// U_S . n_S of interface cell c (all lanes of its group).  U_S = U_P, or with us_mode 1 the
// cell-point interpolation of the velocity to x_S: lane v takes vertex v's velocity with the
// inverse-distance weights of the vertex values; face lane k splits its face about the vertex
// mean into four tetrahedra with the cell centre, carrying U_P, the face's mean vertex velocity
// and the two vertex velocities; each lane keeps the tetrahedron whose smallest barycentric
// coordinate of x_S (Cramer's rule) is largest, and the group takes the best (lowest lane on a
// tie).  Coordinates relative to the vertex mean xm.
template <bool kInterp>
__device__ __forceinline__ double isoface_speed(const SurfArgs &A, int32_t c, int lv, const FaceLane &f,
                                                const int *fv, D3 xm, D3 xS, D3 nS) {
    const DevMesh &m = A.m;
    const size_t n = m.n_cells;
    const D3 Up = vel_at(A.U, A.U1, c, n);
    D3 Us = Up;
    if constexpr (kInterp) {
        D3 uv{0, 0, 0};
        {
            const int k = m.cpt[8 * (size_t)c + lv];
            for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e) uv = uv + m.st_w[e] * vel_at(A.U, A.U1, m.st_cell[e], n);
        }
        D3 uq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) uq[i] = D3{grp_get(uv.x, fv[i]), grp_get(uv.y, fv[i]), grp_get(uv.z, fv[i])};
        const D3 cc = D3{m.ccen[3 * (size_t)c], m.ccen[3 * (size_t)c + 1], m.ccen[3 * (size_t)c + 2]} - xm;
        double best = -INFINITY;
        D3 val = Up;
        if (f.active) {
            // the face's mean point and mean point velocity over its distinct points (a triangle
            // repeats its first point last; its fourth tetrahedron is degenerate and skipped)
            const bool tri = fv[3] == fv[0];
            const D3 fc = tri ? (1.0 / 3.0) * (f.q[0] + f.q[1] + f.q[2]) : 0.25 * (f.q[0] + f.q[1] + f.q[2] + f.q[3]);
            const D3 uf = tri ? (1.0 / 3.0) * (uq[0] + uq[1] + uq[2]) : 0.25 * (uq[0] + uq[1] + uq[2] + uq[3]);
            const D3 e1 = fc - cc, r = xS - cc;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = (i + 1) & 3;
                const D3 e2 = f.q[i] - cc, e3 = f.q[j] - cc;
                const D3 k23 = cross(e2, e3);
                const double det = dot(e1, k23);
                if (det == 0.0) continue;
                const double l1 = dot(r, k23) / det, l2 = dot(e1, cross(r, e3)) / det, l3 = dot(e1, cross(e2, r)) / det;
                const double l0 = 1.0 - l1 - l2 - l3;
                const double mn = fmin(fmin(l0, l1), fmin(l2, l3));
                if (mn > best) {
                    best = mn;
                    val = l0 * Up + l1 * uf + l2 * uq[i] + l3 * uq[j];
                }
            }
        }
        double gb = best;
#pragma unroll
        for (int o = 1; o < kLanes; o <<= 1) gb = fmax(gb, __shfl_xor(gb, o, kLanes));
        const uint64_t bal = __ballot(best == gb);
        const uint32_t gm = (uint32_t)(bal >> (__lane_id() & ~(kLanes - 1))) & 0xFFu;
        const int win = __ffs(gm) - 1;
        Us = D3{grp_get(val.x, win), grp_get(val.y, win), grp_get(val.z, win)};
    }
    return Us.x * nS.x + Us.y * nS.y + Us.z * nS.z;
}


// kMinBlocks: work-groups of 256 per CU the register allocation must allow (waves per SIMD)
// kInterp: U_S by cell-point interpolation (us_mode 1) instead of U_P
// kGeneric: the mesh has cells other than hexahedra (tetrahedra, pyramids, prisms), and every
// cell takes its faces' vertex loops from m.cloop: up to six faces of three or four points (a
// triangle repeats its first point, which gives a zero-length edge that is never cut and adds
// nothing) over up to eight points (lanes past the cell's points repeat its first point).  Cells
// whose faces are all planar take the interval solve like hexahedra (a repeated point adds zero
// terms to the face quadratics and never starts an isoface edge); the others the generic search.
template <int kMinBlocks, bool kInterp, bool kGeneric>
__global__ void __launch_bounds__(256, kMinBlocks) k_surface(SurfArgs A) {
    const DevMesh &m = A.m;
    const int lv = threadIdx.x & (kLanes - 1);
    const int ngrp = (gridDim.x * blockDim.x) / kLanes;
    const int n = min(A.counters[kCntSurf], A.cap);
    // face lv's vertex loop and edge directions (constant per lane on a mesh of hexahedra)
    int fv[4];
    int fwd = lane_face_loop(lv, fv);
    bool face_on = lv < 6;
    int rounds_max = 0, flat = 0, nonconv = 0;
    // groups take list entries round-robin over the XCDs: interface cells are clustered, and
    // contiguous ranges per XCD would leave the XCDs with unequal work
    for (int idx = (blockIdx.x * blockDim.x + threadIdx.x) / kLanes; idx < n; idx += ngrp) {
        const int c = A.list[idx];
        if constexpr (kGeneric) {
            if (m.cbig && m.cbig[c] >= 0) continue;  // a general polyhedron: k_surface_big takes it
            const int32_t L = lv < 6 ? m.cloop[6 * (size_t)c + lv] : 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) fv[i] = (L >> (3 * i)) & 7;
            fwd = (L >> 16) & 15;
            face_on = (L >> 12) & 1;
        }
        const double aP = A.alpha[c];
        const double V6 = 6.0 * m.vol[c];
        const double dtc = cell_dt(m, A.dt_dom, A.dt, c);
        // lane lv: vertex lv's coordinates and value
        const double *cx = m.cxyz + 24 * (size_t)c + 3 * lv;
        D3 xv{cx[0], cx[1], cx[2]};
        double av = 0.0;
        {
            const int k = m.cpt[8 * (size_t)c + lv];
            const int e0 = m.st_ptr[k], e1 = m.st_ptr[k + 1];
            // stencil entries eight at a time: the loads of a chunk are all in flight together
            for (int e = e0; e < e1; e += 8) {
                int32_t sc[8];
                double sw[8], sa[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    sc[j] = e + j < e1 ? m.st_cell[e + j] : -1;
                    sw[j] = e + j < e1 ? m.st_w[e + j] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) sa[j] = sc[j] >= 0 ? A.alpha[sc[j]] : 0.0;
#pragma unroll
                for (int j = 0; j < 8; ++j) av += sw[j] * sa[j];
            }
        }
        if (A.tr.vert_alpha) A.tr.vert_alpha[8 * (size_t)c + lv] = av;
        const D3 xm = 0.125 * grp_sum3(xv);
        xv = xv - xm;
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = grp_get(av, i);
        const bool f_planar = (m.cflags[c] >> min(lv, 5)) & 1;
        // face lv's lane state, built from the group's vertex data; built again after the interval
        // solve rather than held in registers through it
        auto build_face = [&](D3 x, double a) {
            FaceLane r;
            r.active = face_on;
            r.planar = f_planar;
            r.fwd = fwd;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                r.q[i] = D3{grp_get(x.x, fv[i]), grp_get(x.y, fv[i]), grp_get(x.z, fv[i])};
                r.aq[i] = grp_get(a, fv[i]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double d = ((fwd >> i) & 1) ? r.aq[(i + 1) & 3] - r.aq[i] : r.aq[i] - r.aq[(i + 1) & 3];
                r.inv[i] = d != 0.0 ? 1.0 / d : 0.0;
            }
            return r;
        };
        FaceLane f = build_face(xv, av);
        // sorted vertex values (odd-even transposition, 8 elements)
        double s[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = a[i];
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int i = r & 1; i + 1 < 8; i += 2) {
                const double x = fmin(s[i], s[i + 1]), y = fmax(s[i], s[i + 1]);
                s[i] = x;
                s[i + 1] = y;
            }
        bool recon = s[7] - s[0] > A.flat_tol;
        // a hexahedron with six planar faces, or another cell whose faces are all planar
        const bool planar_cell = (m.cflags[c] & 0x13f) == 63 || (kGeneric && (m.cflags[c] & 0x200));
        double iso = 0.0;
        int rounds = 0;
        bool face_done = false;
        D3 nS{0, 0, 0}, xS{0, 0, 0};
        double un = 0.0;
        if (recon) {
            auto F = [&](double x, bool tie_wet) { return cell_vsub6(f, x, tie_wet, nullptr, nullptr) / V6 - aP; };
            auto sorted_at = [&](int i) {
                double r = s[0];
#pragma unroll
                for (int q = 1; q < 8; ++q) r = i == q ? s[q] : r;
                return r;
            };
            // bracket between consecutive sorted vertex values (the sub-volume is smooth in between):
            // the two ends of the guessed interval are probed first, then the search bisects what
            // is left
            int il = 0, ih = 7;
            double fl = 1.0 - aP;
            bool exact = false;
            int p1 = guess_interval<kGeneric>(a, s, aP, lv, !(m.cflags[c] & 0x100)), p2 = p1 + 1;
            while (ih - il > 1) {
                int im = (il + ih) >> 1;
                if (p1 > il && p1 < ih) { im = p1; p1 = -1; }
                else if (p2 > il && p2 < ih) { im = p2; p2 = -1; }
                const double sm = sorted_at(im);
                const double fm = F(sm, false);
                ++rounds;
                if (fm > 0.0) { il = im; fl = fm; }
                else if (fm < 0.0) { ih = im; }
                else { iso = sm; exact = true; break; }
            }
            // planar cells: the interval solve on the face quadratics and isoface edges
            const double lo = sorted_at(il), hi = sorted_at(ih);
            const double xr = 0.5 * (lo + hi);
            double ac[3] = {0.0, 0.0, 0.0};
            Seg sg;
            bool quad = false;
            if (!exact && planar_cell) {
                // wet/dry pattern of the open interval (lo, hi) and the quadratic coefficients
                bool w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = f.aq[i] > xr;
                face_quad_share(f, w, xr, ac);
                quad = spread_edges(face_quad_segs(f, w, xr), lv, sg);
            }
            if (quad) {
                ++rounds;

                // G(u) = six times the sub-volume minus its target, and G'(u): each face adds its
                // wet-loop share plus o(u) . B(u), with o the perimeter centroid of all isoface
                // edges (with no isoface length B vanishes and o does not enter)
                const double target = aP * V6;
                auto G = [&](double u, double &dG) {
                    const Perim pr = seg_eval(sg, u);
                    const D3 oacc = grp_sum3(pr.oacc), doacc = grp_sum3(pr.doacc);
                    const double oL = grp_sum(pr.oL), doL = grp_sum(pr.doL);
                    D3 o{0, 0, 0}, od{0, 0, 0};
                    if (oL > 0.0) {
                        const double il = 1.0 / oL;
                        o = il * oacc;
                        od = il * (doacc - doL * o);
                    }
                    const double gl = ac[0] + u * (ac[1] + u * ac[2]) + dot(o, pr.Bu);
                    const double dgl = ac[1] + 2.0 * u * ac[2] + dot(od, pr.Bu) + dot(o, pr.Bd);
                    dG = grp_sum(dgl);
                    return grp_sum(gl) - target;
                };
                const double ulo = lo - xr, uhi = hi - xr;
                double dG;
                const double gleft = G(uhi, dG);  // the limit from below at hi: pattern w holds there
                if (gleft > 0.0) {
                    iso = hi;  // the sub-volume jumps across alpha_P at this vertex value
                } else {
                    // Newton on G, safeguarded by the bracket [ua, ub] (G(ua) > 0 >= G(ub)).  Where the
                    // root sits next to a bracket end at which the isoface shrinks to a vertex or an
                    // edge, G behaves like a power of the distance to that end and G' vanishes there:
                    // an unusable Newton step is replaced by the root of a cubic power law anchored at
                    // the end with the smaller residual (bisection if that leaves the bracket).
                    double ua = ulo, ub = uhi, ga = fl * V6, gb = gleft;
                    double u = ulo + (uhi - ulo) * (ga / (ga - gb));  // secant start
                    double up = uhi, dGp = dG;  // previous point, for the curvature estimate
                    bool conv = false;
                    for (; rounds < A.max_rounds; ++rounds) {
                        const double g = G(u, dG);
                        if (fabs(g) <= A.root_tol * V6) { conv = true; ++rounds; break; }  // g == 0 at 0
                        if (g > 0.0) { ua = u; ga = g; } else { ub = u; gb = g; }
                        double nu = dG < 0.0 ? u - g / dG : ua;
                        const bool newton = nu > ua && nu < ub;
                        if (!newton) {
                            const bool left = ga <= -gb;
                            const double w = (ub - ua) * cbrt((left ? ga : -gb) / (ga - gb));
                            nu = left ? ua + w : ub - w;
                            if (!(nu > ua && nu < ub)) nu = 0.5 * (ua + ub);
                        }
                        // converged when the step is at round-off of the isovalue, or when a short Newton
                        // step leaves an error |G''| s^2 / (2 |G'|), with G'' from the last two slopes,
                        // below an eighth of that
                        const double tolu = 2.0 * __DBL_EPSILON__ * fmax(fabs(xr + nu), 1e-300);
                        const double s = nu - u;
                        bool done = fabs(s) <= tolu;
                        if (newton && !done && fabs(s) <= 1e-3 * (uhi - ulo))
                            done = fabs(dG - dGp) * s * s <= 0.25 * tolu * fabs(dG) * fabs(u - up);
                        up = u;
                        dGp = dG;
                        u = nu;
                        if (done || !(ub - ua > 2.0 * __DBL_EPSILON__ * fmax(fabs(xr + ua), fabs(xr + ub)))) {
                            conv = true;
                            ++rounds;
                            break;
                        }
                    }
                    if (!conv) ++nonconv;
                    iso = xr + u;
                    // the isoface at the isovalue, from the face segments: apex (perimeter
                    // centroid), area vector (x2) = sum of s x e, centre = area-weighted fan centroid
                    const Perim pr = seg_eval(sg, u);
                    const D3 oacc = grp_sum3(pr.oacc);
                    const double oL = grp_sum(pr.oL);
                    const D3 cs = grp_sum3(pr.Bu);
                    const double nrm = norm3(cs);
                    if (oL > 0.0 && nrm > 0.0) {
                        const D3 o = (1.0 / oL) * oacc;
                        nS = (1.0 / nrm) * cs;
                        const D3 sp = sg.s0 + u * sg.s1, ep = sg.e0 + u * sg.e1;
                        const double wt = sg.on ? dot(cross(sp - o, ep - o), nS) : 0.0;
                        D3 acc = wt * (o + sp + ep);
                        double ws = wt;
                        acc = grp_sum3(acc);
                        ws = grp_sum(ws);
                        xS = (1.0 / (3.0 * ws)) * acc;
                        face_done = true;
                    }
                }
            } else if (!exact) {
                double x0 = sorted_at(il), x1 = sorted_at(ih), f0 = fl;
                double f1 = F(x1, true);  // limit from below at x1
                ++rounds;
                if (f1 > 0.0) {
                    iso = x1;  // the sub-volume jumps across alpha_P at this vertex value
                } else {
                    // Illinois (modified regula falsi) with a bisection guard, to round-off
                    int side = 0;
                    bool conv = false;
                    for (; rounds < A.max_rounds; ++rounds) {
                        const double wdt = x1 - x0;
                        if (!(wdt > 4.0 * __DBL_EPSILON__ * fmax(fabs(x0), fabs(x1)))) { conv = true; break; }
                        double x = x1 - f1 * (x1 - x0) / (f1 - f0);
                        if (!(x > x0 && x < x1) || (rounds & 7) == 7) x = x0 + 0.5 * wdt;
                        const double fx = F(x, false);
                        if (fabs(fx) <= fmax(4.0 * __DBL_EPSILON__, A.root_tol)) {
                            x0 = x1 = x;
                            f0 = f1 = fx;
                            conv = true;
                            ++rounds;
                            break;
                        }
                        if (fx > 0.0) {
                            x0 = x; f0 = fx;
                            if (side == 1) f1 *= 0.5;
                            side = 1;
                        } else {
                            x1 = x; f1 = fx;
                            if (side == -1) f0 *= 0.5;
                            side = -1;
                        }
                    }
                    if (!conv) ++nonconv;
                    iso = fabs(f0) <= fabs(f1) ? x0 : x1;
                }
            }
            if (quad) {
                // the same values again: the empty asm hides that, so that the first copy need not
                // stay live through the solve
                D3 x2 = xv;
                double a2 = av;
                asm volatile("" : "+v"(x2.x), "+v"(x2.y), "+v"(x2.z), "+v"(a2));
                f = build_face(x2, a2);
            }
            // isoface at the isovalue (unless the interval solve already built it)
            D3 o, cseg{0, 0, 0};
            if (!face_done) cell_vsub6(f, iso, false, &o, &cseg);
            const double nrm = norm3(cseg);
            if (face_done) {
            } else if (nrm > 0.0) {
                nS = (1.0 / nrm) * cseg;
                D3 acc;
                double ws;
                face_centre_part(f, iso, o, nS, acc, ws);
                acc = grp_sum3(acc);
                ws = grp_sum(ws);
                xS = (1.0 / (3.0 * ws)) * acc;
            } else {
                recon = false;
            }
        }
        if (recon) un = isoface_speed<kInterp>(A, c, lv, f, fv, xm, xS, nS);
        if (lv == 0) {
            if (!recon) ++flat;
            rounds_max = max(rounds_max, rounds);
            if (A.tr.kind) A.tr.kind[c] = recon ? 1 : 2;
            if (recon) {
                if (A.tr.iso) A.tr.iso[c] = iso;
                if (A.tr.iters) A.tr.iters[c] = rounds;
                if (A.tr.rec) {
                    double *rr = A.tr.rec + 7 * (size_t)c;
                    rr[0] = xS.x + xm.x; rr[1] = xS.y + xm.y; rr[2] = xS.z + xm.z;
                    rr[3] = nS.x; rr[4] = nS.y; rr[5] = nS.z; rr[6] = un;
                }
            }
            if (!recon) (void)nonconv;
        }
        // lane k < 6: face k, if it is an outflow face of this cell
        if (f.active) {
            const int32_t v = m.lface[6 * (size_t)c + lv];
            if (v != kEmpty) {
                const int32_t fid = v >= 0 ? v : ~v;
                const double ph = A.phi1 ? flux_at<true>(A.phi, A.phi1, fid) : flux_at<false>(A.phi, A.phi1, fid);
                const double out = v >= 0 ? ph : -ph;
                if (out > 0.0) {
                    double dv;
                    if (recon) {
                        double dq[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = dot(f.q[i] - xS, nS);
                        double acc = 0.0, Af = 0.0;
                        if (f.planar) {
                            // planar face: two triangles cover it exactly
                            const double A1 = 0.5 * norm3(cross(f.q[1] - f.q[0], f.q[2] - f.q[0]));
                            const double A2 = 0.5 * norm3(cross(f.q[2] - f.q[0], f.q[3] - f.q[0]));
                            acc = A1 * tri_sweep(dq[0], dq[1], dq[2], un, dtc) +
                                  A2 * tri_sweep(dq[0], dq[2], dq[3], un, dtc);
                            Af = A1 + A2;
                        } else {
                            // fan about the vertex mean
                            const D3 ap = 0.25 * (f.q[0] + f.q[1] + f.q[2] + f.q[3]);
                            const double dap = dot(ap - xS, nS);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const double Ai = 0.5 * norm3(cross(f.q[i] - ap, f.q[(i + 1) & 3] - ap));
                                acc += Ai * tri_sweep(dap, dq[i], dq[(i + 1) & 3], un, dtc);
                                Af += Ai;
                            }
                        }
                        dv = ph * (acc / Af);
                    } else {
                        dv = aP * ph * dtc;
                    }
                    A.dvs[fid] = dv;
                }
            }
        }
    }
    if (A.want_stats) {
        for (int off = 32; off > 0; off >>= 1) {
            rounds_max = max(rounds_max, __shfl_xor(rounds_max, off));
            flat += __shfl_xor(flat, off);
            nonconv += __shfl_xor(nonconv, off);
        }
        if (__lane_id() == 0) {
            if (rounds_max) atomicMax(&A.counters[kCntMaxIter], rounds_max);
            if (flat) atomicAdd(&A.counters[kCntFlat], flat);
            if (nonconv) atomicAdd(&A.counters[kCntNonconv], nonconv / kLanes);
        }
    }
}

struct UpdArgs {
    DevMesh m;
    const double *alpha, *phi, *dvs;
    double dt;
    const double *dt_dom;
    double eps, tol;
    int clip;
    double *alpha_new;
    int32_t *olist;
    int32_t *counters;
    double *trace_dV, *trace_raw;
    int n_iter;  // redistribution sweeps; with one or more the update runs the first sweep's phase A
    DevWork w;
    const double *phi1;  // second time level of the fluxes, or nullptr
    int stats;  // per-cell volume through boundary faces and clipped volume into w.sbnd, w.sclip
};

// Bounding counters of sweep `it` live in one of four rotating slots: a slot is filled by the
// kernel before its sweep's (phase A), read by its sweep's kernel and the next one, and cleared by
// the one after that.
__device__ __forceinline__ int32_t *bound_slot(int32_t *counters, int it) { return counters + kCntBound + 2 * (it % 4); }
enum : int { kSlotTouched = 0, kSlotDelta = 1 };

// Sweep s's corrections and their face list: three rotating buffers, so that a kernel can apply
// sweep s, compute sweep s+1 and clear what sweep s-1 left, all on different buffers.
__device__ __forceinline__ double *delta_buf(const DevWork &w, int s, int nf) { return w.delta + (size_t)(s % 3) * nf; }
__device__ __forceinline__ int32_t *dlist_buf(const DevWork &w, int s, int nf) {
    return w.flist + (size_t)(1 + s % 3) * nf;
}

// W flux slots per cell, all loads of one kind issued together (independent gathers in flight).
// Any block size up to 1024 (the block_cells option) is valid.  A cell left out of bounds also
// runs phase A of the first redistribution sweep (see k_bound_sweep) here: no face is marked yet,
// so the current dV of each of its outflow faces is the one just computed.
template <int W, bool kAvg, bool kDom>
__global__ void __launch_bounds__(1024) k_update(UpdArgs A) {
    // no fused multiply-adds: the single-mesh and ensemble instantiations then round every
    // operation alike, and an ensemble member gets the same bits as the member stepped alone
#pragma clang fp contract(off)
    const int n = A.m.n_cells;
    const int c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    bool offend = false;
    int32_t v[W], o[W];
    double ph[W], dvo[W];  // face fluxes; dV of the outflow faces (0 elsewhere)
    double x = 0.0, V = 0.0, dtc = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        v[k] = kEmpty;
        o[k] = -1;
        ph[k] = dvo[k] = 0.0;
    }
    if (c < n) {
        int dom = -1;  // the ensemble member, when the slot words have given it
        if (A.m.slot_nar) {
            // the 32-bit slot words: all loaded before any is decoded, then the slots they send
            // to the full tables
            uint32_t wd[W];
            bool wide[W];
#pragma unroll
            for (int k = 0; k < W; ++k) wd[k] = __builtin_nontemporal_load(A.m.slot_nar + (size_t)k * n + c);
            auto decode = [&](uint32_t S, int32_t c0, int32_t f0) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const uint32_t h = wd[k] & 0xFFFFu;
                    const int32_t up = (int32_t)(int16_t)(uint16_t)(wd[k] >> 16);
                    const int32_t nb = c + (up >= 0 ? up + 1 : up);
                    const uint32_t owner = (uint32_t)(min(c, nb) - c0);
                    const int32_t f = f0 + (int32_t)(((uint64_t)owner * S) >> 28) + (int32_t)h;
                    wide[k] = h == 0xFFFFu;
                    v[k] = h == 0xFFFEu ? kEmpty : (c < nb ? f : ~f);
                    o[k] = h == 0xFFFEu ? -1 : nb;
                }
            };
            if constexpr (kDom) {
                // the member's constants from the record of the cell's 64-cell block
                const int4 *rec = reinterpret_cast<const int4 *>(A.m.nar_blk) + 2 * (size_t)(c >> 6);
                const int4 ra = rec[0], rb = rec[1];
                if (ra.w < 0) {
                    dom = cell_dom(A.m, c);
                    decode((uint32_t)A.m.nar_dom[3 * dom], A.m.nar_dom[3 * dom + 2], A.m.nar_dom[3 * dom + 1]);
                } else if ((c & 63) >= ra.w) {
                    dom = rb.w + 1;
                    decode((uint32_t)rb.x, rb.z, rb.y);
                } else {
                    dom = rb.w;
                    decode((uint32_t)ra.x, ra.z, ra.y);
                }
            } else {
                decode(A.m.nar_S, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (wide[k]) {
                    v[k] = __builtin_nontemporal_load(A.m.slot_face + (size_t)k * n + c);
                    o[k] = __builtin_nontemporal_load(A.m.slot_nbr + (size_t)k * n + c);
                }
        } else {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                v[k] = __builtin_nontemporal_load(A.m.slot_face + (size_t)k * n + c);
                o[k] = __builtin_nontemporal_load(A.m.slot_nbr + (size_t)k * n + c);
            }
        }
        const double aP = A.alpha[c];
        V = __builtin_nontemporal_load(A.m.vol + c);
        double ao[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int32_t fid = v[k] >= 0 ? v[k] : ~v[k];
            ph[k] = v[k] != kEmpty ? flux_at<kAvg>(A.phi, A.phi1, fid) : 0.0;
            ao[k] = o[k] >= 0 ? A.alpha[o[k]] : (v[k] != kEmpty ? A.m.patch_alpha[-1 - o[k]] : 0.0);
        }
        const bool sP = interface_cell(aP, A.eps);
        if constexpr (kDom) dtc = dom >= 0 ? A.dt_dom[dom] : cell_dt(A.m, A.dt_dom, A.dt, c);
        else dtc = cell_dt(A.m, A.dt_dom, A.dt, c);
        double sum = 0.0, bnd = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (v[k] == kEmpty) continue;
            const int32_t fid = v[k] >= 0 ? v[k] : ~v[k];
            const double out = v[k] >= 0 ? ph[k] : -ph[k];
            double dv = 0.0;
            if (out > 0.0) {
                dv = sP ? A.dvs[fid] : aP * ph[k] * dtc;
                dvo[k] = dv;
            } else if (out < 0.0) {
                dv = (o[k] >= 0 && interface_cell(ao[k], A.eps)) ? A.dvs[fid] : ao[k] * ph[k] * dtc;
            }
            sum += v[k] >= 0 ? dv : -dv;
            if (o[k] < 0) bnd += dv;  // a boundary face: the cell owns it
            if (A.trace_dV && v[k] >= 0) A.trace_dV[fid] = dv;
        }
        x = aP - sum / V;
        if (A.trace_raw) A.trace_raw[c] = x;
        const double x0 = x;
        if (A.clip) {
            if (x < 0.0 && x >= -A.tol) x = 0.0;
            else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
        }
        if (A.stats) {
            A.w.sbnd[c] = bnd;
            A.w.sclip[c] = (x - x0) * V;
        }
        offend = x > 1.0 + A.tol || x < -A.tol;
        A.alpha_new[c] = x;  // a plain store: the next step's find kernel reads it from the caches
    }
    const uint64_t mask = __ballot(offend);
    if (mask == 0) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&A.counters[kCntOff], __popcll(mask));
    base = __shfl(base, leader);
    if (offend)
        A.olist[base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))] = c;
    if (A.n_iter < 1) return;
    // phase A of sweep 0 (as in k_bound_sweep, with every face unmarked)
    const int nf = A.m.n_faces;
    int32_t *slot = bound_slot(A.counters, 0);
    int ndl = 0, ntl = 0;
    int32_t fsel[W], tsel[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) tsel[k] = -1;
#pragma unroll
    for (int k = 0; k < W; ++k) fsel[k] = -1;
    if (offend) {
        const bool over = x > 1.0 + A.tol;
        double cap[W];
        double sumcap = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            cap[k] = 0.0;
            if (v[k] == kEmpty) continue;
            const double outphi = v[k] >= 0 ? ph[k] : -ph[k];
            if (!(outphi > 0.0)) continue;
            const double outv = v[k] >= 0 ? dvo[k] : -dvo[k];
            cap[k] = over ? outphi * dtc - outv : outv;
            if (cap[k] > 0.0) sumcap += cap[k];
        }
        if (atomicExch(&A.w.cmark[c], 1) == 0) tsel[W] = c;
        const double need = over ? (x - 1.0) * V : -x * V;
        const double r = sumcap > 0.0 ? fmin(need / sumcap, 1.0) : 0.0;
        double bcorr = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (!(sumcap > 0.0) || !(cap[k] > 0.0)) continue;
            const double d = cap[k] * r;
            const double dd = over ? (v[k] >= 0 ? d : -d) : (v[k] >= 0 ? -d : d);
            const int32_t f = v[k] >= 0 ? v[k] : ~v[k];
            delta_buf(A.w, 0, nf)[f] = dd;
            A.w.dvcur[f] = dvo[k] + dd;
            A.w.fmark[f] = 1;
            fsel[k] = f;
            if (o[k] >= 0 && atomicExch(&A.w.cmark[o[k]], 1) == 0) tsel[k] = o[k];
            if (o[k] < 0) bcorr += dd;
        }
        if (A.stats && bcorr != 0.0) A.w.sbnd[c] += bcorr;
#pragma unroll
        for (int k = 0; k < W; ++k) ndl += fsel[k] >= 0 ? 1 : 0;
#pragma unroll
        for (int k = 0; k <= W; ++k) ntl += tsel[k] >= 0 ? 1 : 0;
    }
    // every marked face is new at sweep 0: it enters both the sweep's correction list and flist
    int bd = wave_append(ndl, &slot[kSlotDelta]);
    int bf = wave_append(ndl, &A.counters[kCntFaces]);
    int bt = wave_append(ntl, &slot[kSlotTouched]);
    int32_t *dlist = dlist_buf(A.w, 0, nf);
#pragma unroll
    for (int k = 0; k < W; ++k)
        if (fsel[k] >= 0) {
            dlist[bd++] = fsel[k];
            A.w.flist[bf++] = fsel[k];
        }
#pragma unroll
    for (int k = 0; k <= W; ++k)
        if (tsel[k] >= 0) A.w.tlist[bt++] = tsel[k];
}

struct BoundArgs {
    DevMesh m;
    const double *alpha, *phi, *dvs;
    double dt;
    const double *dt_dom;
    double eps, tol;
    int clip, n_iter;
    double *alpha_new;
    DevWork w;
    const double *phi1;  // second time level of the fluxes, or nullptr
    int stats;  // add the sweeps' boundary-face corrections and clipped volumes to w.sbnd, w.sclip
};

// Redistribution sweeps (Jacobi), two phases per sweep.  (A) every cell out of bounds computes the
// change of the heavy-fluid outflow of each of its outflow faces (each face has one upwind cell,
// so it alone writes that face's correction and its running dV) and marks the cells it touches;
// (B) every touched cell applies the corrections of its faces in ascending face order.  Phase A
// of a cell needs only its own new alpha and its own outflow faces, so a cell still out of bounds
// after phase B of sweep s runs phase A of sweep s+1 at once: one kernel per sweep (phase A of
// sweep 0 runs inside the update).  Touched lists and marks alternate between two banks, counter
// slots rotate over four.  List order never affects a result.
template <int W, bool kAvg>
__global__ void __launch_bounds__(256) k_bound_sweep(BoundArgs A, int it) {
    const int n = A.m.n_cells, nf = A.m.n_faces;
    int32_t *counters = A.w.counters;
    const int stride = gridDim.x * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    const bool last = it == A.n_iter - 1;
    if (it >= 1) {  // sweep it-1's corrections were read by the previous kernel: clear them
        const int n_stale = bound_slot(counters, it - 1)[kSlotDelta];
        double *stale = delta_buf(A.w, it - 1, nf);
        const int32_t *slist = dlist_buf(A.w, it - 1, nf);
        for (int i = t0; i < n_stale; i += stride) stale[slist[i]] = 0.0;
    }
    // nothing reads sweep it-2's counters any more (its slot returns for sweep it+2)
    if (it >= 2 && blockIdx.x == 0 && threadIdx.x < 2) bound_slot(counters, it - 2)[threadIdx.x] = 0;
    const int32_t *slot = bound_slot(counters, it);
    int32_t *slot_next = bound_slot(counters, it + 1);
    const double *delta = delta_buf(A.w, it, nf);
    double *delta_next = delta_buf(A.w, it + 1, nf);
    int32_t *dlist_next = dlist_buf(A.w, it + 1, nf);
    const int32_t *touched = A.w.tlist + (size_t)(it & 1) * n;
    int32_t *touched_next = A.w.tlist + (size_t)((it + 1) & 1) * n;
    int32_t *mark = A.w.cmark + (size_t)(it & 1) * n;
    int32_t *mark_next = A.w.cmark + (size_t)((it + 1) & 1) * n;
    const int nT = slot[kSlotTouched];
    if (last) {
        // no phase A in the last sweep reads the face marks, and the list of marked faces is
        // complete: clear them here, over the whole grid, rather than in the end kernel
        const int nF = counters[kCntFaces];
        for (int i = t0; i < nF; i += stride) A.w.fmark[A.w.flist[i]] = 0;
    }
    const int nloop = (nT + 255) & ~255;  // whole work-groups iterate together
    for (int i0 = blockIdx.x * blockDim.x; i0 < nloop; i0 += stride) {
        const int i = i0 + threadIdx.x;
        bool again = false;
        int32_t Q = 0;
        double x = 0.0;
        int32_t v[W], nb[W];
        // phase B of sweep it
        if (i < nT) {
            Q = touched[i];
            const int2 *sp = A.m.slot_pair + (size_t)Q * W;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int2 q = sp[k];
                v[k] = q.x;
                nb[k] = q.y;
            }
            const double aq = A.alpha_new[Q], vq = A.m.vol[Q];
            double d[W];
#pragma unroll
            for (int k = 0; k < W; ++k) d[k] = v[k] != kEmpty ? delta[v[k] >= 0 ? v[k] : ~v[k]] : 0.0;
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (v[k] != kEmpty) sum += v[k] >= 0 ? d[k] : -d[k];
            x = aq - sum / vq;
            const double xb = x;
            if (A.clip) {
                if (x < 0.0 && x >= -A.tol) x = 0.0;
                else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
                if (last) x = fmin(fmax(x, 0.0), 1.0);
            }
            if (A.stats && x != xb) A.w.sclip[Q] += (x - xb) * vq;
            A.alpha_new[Q] = x;
            mark[Q] = 0;
            again = x > 1.0 + A.tol || x < -A.tol;
        }
        if (last) continue;  // uniform
        // phase A of sweep it+1 for a cell still out of bounds
        int ndl = 0, nfl = 0, ntl = 0;
        int32_t fsel[W], tsel[W + 1];
        bool newf[W];
#pragma unroll
        for (int k = 0; k < W; ++k) { fsel[k] = -1; newf[k] = false; tsel[k] = -1; }
        tsel[W] = -1;
        if (again) {
            int32_t nbr[W], fid[W];
            double ph[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                nbr[k] = nb[k];
                fid[k] = v[k] >= 0 ? v[k] : ~v[k];
                ph[k] = v[k] != kEmpty ? flux_at<kAvg>(A.phi, A.phi1, fid[k]) : 0.0;
            }
            const bool over = x > 1.0 + A.tol;
            const double aold = A.alpha[Q];
            const bool sP = interface_cell(aold, A.eps);
            const double dtc = cell_dt(A.m, A.dt_dom, A.dt, Q);
            int32_t mk[W];
            double dvs_v[W], dvc_v[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const bool outflow = v[k] != kEmpty && (v[k] >= 0 ? ph[k] : -ph[k]) > 0.0;
                mk[k] = outflow ? A.w.fmark[fid[k]] : 0;
                dvs_v[k] = (outflow && sP) ? A.dvs[fid[k]] : 0.0;
                dvc_v[k] = outflow ? A.w.dvcur[fid[k]] : 0.0;
            }
            double cap[W], dvnow[W];
            double sumcap = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                cap[k] = 0.0;
                dvnow[k] = 0.0;
                if (v[k] == kEmpty) continue;
                const double outphi = v[k] >= 0 ? ph[k] : -ph[k];
                if (!(outphi > 0.0)) continue;
                // current dV of the face: running value once touched, else this step's
                dvnow[k] = mk[k] ? dvc_v[k] : (sP ? dvs_v[k] : aold * ph[k] * dtc);
                const double outv = v[k] >= 0 ? dvnow[k] : -dvnow[k];
                cap[k] = over ? outphi * dtc - outv : outv;
                if (cap[k] > 0.0) sumcap += cap[k];
            }
            if (atomicExch(&mark_next[Q], 1) == 0) tsel[W] = Q;
            const double need = over ? (x - 1.0) * A.m.vol[Q] : -x * A.m.vol[Q];
            const double r = sumcap > 0.0 ? fmin(need / sumcap, 1.0) : 0.0;
            double bcorr = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                if (!(sumcap > 0.0) || !(cap[k] > 0.0)) continue;
                const double dk = cap[k] * r;
                const double dd = over ? (v[k] >= 0 ? dk : -dk) : (v[k] >= 0 ? -dk : dk);
                const int32_t f = fid[k];
                delta_next[f] = dd;
                A.w.dvcur[f] = dvnow[k] + dd;
                fsel[k] = f;
                if (!mk[k]) {
                    A.w.fmark[f] = 1;
                    newf[k] = true;
                }
                if (nbr[k] >= 0 && atomicExch(&mark_next[nbr[k]], 1) == 0) tsel[k] = nbr[k];
                if (nbr[k] < 0) bcorr += dd;
            }
            if (A.stats && bcorr != 0.0) A.w.sbnd[Q] += bcorr;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                ndl += fsel[k] >= 0 ? 1 : 0;
                nfl += newf[k] ? 1 : 0;
            }
#pragma unroll
            for (int k = 0; k <= W; ++k) ntl += tsel[k] >= 0 ? 1 : 0;
        }
        int bd = wave_append(ndl, &slot_next[kSlotDelta]);
        int bf = wave_append(nfl, &counters[kCntFaces]);
        int bt = wave_append(ntl, &slot_next[kSlotTouched]);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (fsel[k] >= 0) dlist_next[bd++] = fsel[k];
            if (newf[k]) A.w.flist[bf++] = fsel[k];
        }
#pragma unroll
        for (int k = 0; k <= W; ++k)
            if (tsel[k] >= 0) touched_next[bt++] = tsel[k];
    }
}

// End of the step (one work-group): chop the listed cells when no sweep ran, clear the correction
// buffer of the last sweep (the last sweep itself has cleared the face marks), keep this step's
// counters for the statistics and zero them for the next step.
__global__ void __launch_bounds__(1024) k_bound_end(BoundArgs A) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nf = A.m.n_faces;
    int32_t *counters = A.w.counters;
    if (A.n_iter == 0) {
        if (A.clip) {
            const int nO = counters[kCntOff];
            for (int i = tid; i < nO; i += nt) {
                const int32_t P = A.w.olist[i];
                const double x = A.alpha_new[P], y = fmin(fmax(x, 0.0), 1.0);
                A.alpha_new[P] = y;
                if (A.stats) A.w.sclip[P] += (y - x) * A.m.vol[P];
            }
        }
    } else {
        const int it = A.n_iter - 1;
        const int nd = bound_slot(counters, it)[kSlotDelta];
        const int32_t *dl = dlist_buf(A.w, it, nf);
        double *delta = delta_buf(A.w, it, nf);
        for (int i = tid; i < nd; i += nt) delta[dl[i]] = 0.0;
    }
    if (A.n_iter == 0) {  // (with sweeps, the last one has cleared the face marks)
        const int nF = counters[kCntFaces];
        for (int i = tid; i < nF; i += nt) A.w.fmark[A.w.flist[i]] = 0;
    }
    __syncthreads();
    if (tid < 8) counters[8 + tid] = tid == kCntActive0 ? counters[kCntOff] : counters[tid];
    __syncthreads();
    if (tid < 8) counters[tid] = 0;
    if (tid >= kCntBound && tid < kCntBound + 8) counters[tid] = 0;
}

// Step statistics in two passes with a fixed order of summation (results do not depend on timing):
// work-group b reduces the cells [b chunk, (b + 1) chunk) to six partial values, one work-group
// then reduces those: volume before and after, smallest and largest alpha, clipped volume and the
// volume that left through the boundary.
constexpr int kStatBlocks = 256, kStatThreads = 256, kStatVals = 6;

__device__ __forceinline__ void stat_reduce(double (&v)[kStatVals], double (*sh)[kStatThreads]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kStatVals; ++i) sh[i][t] = v[i];
    __syncthreads();
    for (int h = kStatThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            sh[0][t] += sh[0][t + h];
            sh[1][t] += sh[1][t + h];
            sh[2][t] = fmin(sh[2][t], sh[2][t + h]);
            sh[3][t] = fmax(sh[3][t], sh[3][t + h]);
            sh[4][t] += sh[4][t + h];
            sh[5][t] += sh[5][t + h];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kStatThreads) k_stats_part(const double *alpha, const double *alpha_new,
                                                           const double *vol, const double *sclip,
                                                           const double *sbnd, int n, double *part) {
    __shared__ double sh[kStatVals][kStatThreads];
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int c0 = blockIdx.x * chunk, c1 = min(n, c0 + chunk);
    double v[kStatVals] = {0.0, 0.0, 1e300, -1e300, 0.0, 0.0};
    for (int c = c0 + (int)threadIdx.x; c < c1; c += kStatThreads) {
        const double V = vol[c], an = alpha_new[c];
        v[0] += alpha[c] * V;
        v[1] += an * V;
        v[2] = fmin(v[2], an);
        v[3] = fmax(v[3], an);
        v[4] += sclip[c];
        v[5] += sbnd[c];
    }
    stat_reduce(v, sh);
    if (threadIdx.x < kStatVals) part[kStatVals * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(kStatThreads) k_stats_final(const double *part, int nb, double *red) {
    __shared__ double sh[kStatVals][kStatThreads];
    double v[kStatVals] = {0.0, 0.0, 1e300, -1e300, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kStatThreads) {
        const double *q = part + kStatVals * b;
        v[0] += q[0];
        v[1] += q[1];
        v[2] = fmin(v[2], q[2]);
        v[3] = fmax(v[3], q[3]);
        v[4] += q[4];
        v[5] += q[5];
    }
    stat_reduce(v, sh);
    if (threadIdx.x < kStatVals) red[threadIdx.x] = sh[threadIdx.x][0];
}

template <int W, bool kAvg>
void launch_wide(const DevMesh &m, const UpdArgs &ua, const BoundArgs &ba, const LaunchCfg &cfg, hipStream_t s,
                 hipEvent_t *ev) {
    const int gc = (m.n_cells + cfg.block_cells - 1) / cfg.block_cells;
    // and sweep 0's phase A; ensembles take the members' constants and time steps per cell
    if (m.n_dom > 0) hipLaunchKernelGGL((k_update<W, kAvg, true>), dim3(gc), dim3(cfg.block_cells), 0, s, ua);
    else hipLaunchKernelGGL((k_update<W, kAvg, false>), dim3(gc), dim3(cfg.block_cells), 0, s, ua);
    if (ev) (void)hipEventRecord(ev[3], s);
    for (int it = 0; it < ba.n_iter; ++it)
        hipLaunchKernelGGL((k_bound_sweep<W, kAvg>), dim3(cfg.bound_blocks), dim3(256), 0, s, ba, it);
    hipLaunchKernelGGL(k_bound_end, dim3(1), dim3(1024), 0, s, ba);
}

__global__ void k_offset_copy(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int64_t n, int mode,
                              int32_t off1, int32_t off2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!src) { dst[i] = off1; continue; }
        const int32_t v = src[i];
        int32_t r;
        if (mode == 0) r = v >= 0 ? v + off1 : v;
        else if (mode == 1) r = v == kEmpty ? v : (v >= 0 ? v + off1 : ~(~v + off1));
        else r = v >= 0 ? v + off1 : -1 - (-1 - v + off2);
        dst[i] = r;
    }
}

__global__ void k_slot_pairs(DevMesh m, int2 *__restrict__ pairs) {
    const int n = m.n_cells, W = m.W;
    const int64_t tot = (int64_t)n * W;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / W), k = (int)(t % W);
        pairs[t] = make_int2(m.slot_face[(size_t)k * n + c], m.slot_nbr[(size_t)k * n + c]);
    }
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_step(const DevMesh &m, const DevWork &w, const Params &p, const StepArgs &a, const iso_trace *trace,
                       const LaunchCfg &cfg, bool want_stats, hipStream_t s, hipEvent_t *ev) {
    // launch shapes must stay within what each kernel was compiled for
    if (cfg.block_cells < 1 || cfg.block_cells > 1024 || cfg.surface_blocks < 0 || cfg.surface_blocks > 65535 ||
        cfg.surface_waves < 1 || cfg.surface_waves > 4 || cfg.bound_blocks < 1 || cfg.bound_blocks > 65535)
        return hipErrorInvalidValue;
    const int n = m.n_cells;
    iso_trace tr{};
    if (trace) tr = *trace;
    if (ev) (void)hipEventRecord(ev[0], s);
    const int gf = (int)(((size_t)n + kFindBlock * kFindPerThread - 1) / (kFindBlock * kFindPerThread));
    hipLaunchKernelGGL(k_find_surface, dim3(gf), dim3(kFindBlock), 0, s, a.alpha, n, p.eps_surf, w.surf, w.cap,
                       w.counters, tr.kind);
    if (ev) (void)hipEventRecord(ev[1], s);
    SurfArgs sa{m, a.alpha, a.phi, a.U, a.dt, a.dt_dom, p.eps_surf, p.flat_tol, p.root_max_iter, w.surf, w.counters,
                w.cap, w.dvs, want_stats ? 1 : 0, tr, a.phi1, a.U1, p.root_tol};
    const int bs = 256;  // the interface kernel's register budget assumes 256-thread work-groups
    const long groups_per_block = bs / kLanes;
    long gs = ((long)w.cap + groups_per_block - 1) / groups_per_block;
    // persistent: groups loop over the list, which is only known on the device
    gs = std::max(1L, std::min(gs, cfg.surface_blocks > 0 ? (long)cfg.surface_blocks : 2048L));
    if (m.cbig) {  // general polyhedra: their kernel on the side stream, beside the eight-lane one
        hipStream_t sb = s;
        if (w.side) {
            hipError_t e = hipEventRecord(w.fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(w.side, w.fork, 0);
            if (e != hipSuccess) return e;
            sb = w.side;
        }
        BigArgs bg{m, a.alpha, a.phi, a.U, a.phi1, a.U1, a.dt, p.flat_tol, p.root_max_iter, a.dt_dom, w.surf,
                   w.counters, w.cap, w.dvs, want_stats ? 1 : 0, tr, p.root_tol, p.us_mode};
        const hipError_t e = launch_surface_big(bg, sb);
        if (e != hipSuccess) return e;
    }
    if (m.all_big) {
        // every cell is taken by the polyhedron kernel: nothing for the eight-lane one
    } else if (m.cloop && p.us_mode == 0) {
        switch (cfg.surface_waves) {
            case 1: hipLaunchKernelGGL((k_surface<1, false, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 3: hipLaunchKernelGGL((k_surface<3, false, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 4: hipLaunchKernelGGL((k_surface<4, false, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            default: hipLaunchKernelGGL((k_surface<2, false, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
        }
    } else if (m.cloop && p.us_mode == 1) {
        switch (cfg.surface_waves) {
            case 1: hipLaunchKernelGGL((k_surface<1, true, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 3: hipLaunchKernelGGL((k_surface<3, true, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 4: hipLaunchKernelGGL((k_surface<4, true, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            default: hipLaunchKernelGGL((k_surface<2, true, true>), dim3((int)gs), dim3(bs), 0, s, sa); break;
        }
    } else if (p.us_mode == 1) {
        switch (cfg.surface_waves) {
            case 1: hipLaunchKernelGGL((k_surface<1, true, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 3: hipLaunchKernelGGL((k_surface<3, true, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 4: hipLaunchKernelGGL((k_surface<4, true, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            default: hipLaunchKernelGGL((k_surface<2, true, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
        }
    } else {
        switch (cfg.surface_waves) {
            case 1: hipLaunchKernelGGL((k_surface<1, false, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 3: hipLaunchKernelGGL((k_surface<3, false, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            case 4: hipLaunchKernelGGL((k_surface<4, false, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
            default: hipLaunchKernelGGL((k_surface<2, false, false>), dim3((int)gs), dim3(bs), 0, s, sa); break;
        }
    }
    if (m.cbig && w.side) {
        hipError_t e = hipEventRecord(w.join, w.side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, w.join, 0);
        if (e != hipSuccess) return e;
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    const int st = want_stats && w.sbnd && w.sclip ? 1 : 0;
    UpdArgs ua{m, a.alpha, a.phi, w.dvs, a.dt, a.dt_dom, p.eps_surf, p.bound_tol, p.clip, a.alpha_new, w.olist,
               w.counters, tr.dV, tr.alpha_raw, p.n_bound_iter, w, a.phi1, st};
    if (!cfg.compact_slots) ua.m.slot_nar = nullptr;
    BoundArgs ba{m, a.alpha, a.phi, w.dvs, a.dt, a.dt_dom, p.eps_surf, p.bound_tol, p.clip, p.n_bound_iter,
                 a.alpha_new, w, a.phi1, st};
    const bool avg = a.phi1 != nullptr;
    // more than six flux faces (general polyhedra): the plan pads the slots to width 8, 12 or 16
    switch (m.W * 2 + (avg ? 1 : 0)) {
        case 2: launch_wide<1, false>(m, ua, ba, cfg, s, ev); break;
        case 3: launch_wide<1, true>(m, ua, ba, cfg, s, ev); break;
        case 4: launch_wide<2, false>(m, ua, ba, cfg, s, ev); break;
        case 5: launch_wide<2, true>(m, ua, ba, cfg, s, ev); break;
        case 6: launch_wide<3, false>(m, ua, ba, cfg, s, ev); break;
        case 7: launch_wide<3, true>(m, ua, ba, cfg, s, ev); break;
        case 8: launch_wide<4, false>(m, ua, ba, cfg, s, ev); break;
        case 9: launch_wide<4, true>(m, ua, ba, cfg, s, ev); break;
        case 10: launch_wide<5, false>(m, ua, ba, cfg, s, ev); break;
        case 11: launch_wide<5, true>(m, ua, ba, cfg, s, ev); break;
        case 13: launch_wide<6, true>(m, ua, ba, cfg, s, ev); break;
        case 16: launch_wide<8, false>(m, ua, ba, cfg, s, ev); break;
        case 17: launch_wide<8, true>(m, ua, ba, cfg, s, ev); break;
        case 24: launch_wide<12, false>(m, ua, ba, cfg, s, ev); break;
        case 25: launch_wide<12, true>(m, ua, ba, cfg, s, ev); break;
        case 32: launch_wide<16, false>(m, ua, ba, cfg, s, ev); break;
        case 33: launch_wide<16, true>(m, ua, ba, cfg, s, ev); break;
        default: launch_wide<6, false>(m, ua, ba, cfg, s, ev); break;
    }
    if (ev) (void)hipEventRecord(ev[4], s);
    return hipGetLastError();
}

hipError_t launch_offset_copy(const int32_t *src, int32_t *dst, int64_t n, int mode, int32_t off1, int32_t off2,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_offset_copy, dim3(g), dim3(256), 0, s, src, dst, n, mode, off1, off2);
    return hipGetLastError();
}

hipError_t launch_slot_pairs(const DevMesh &m, int2 *pairs, hipStream_t s) {
    const int64_t n = (int64_t)m.n_cells * m.W;
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_slot_pairs, dim3(g), dim3(256), 0, s, m, pairs);
    return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_stats(const DevMesh &m, const DevWork &w, const double *alpha, const double *alpha_new,
                        hipStream_t s) {
    // partial values after the eight results (the host copies red[0, 8))
    hipLaunchKernelGGL(k_stats_part, dim3(kStatBlocks), dim3(kStatThreads), 0, s, alpha, alpha_new, m.vol, w.sclip,
                       w.sbnd, m.n_cells, w.red + 8);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kStatThreads), 0, s, w.red + 8, kStatBlocks, w.red);
    return hipGetLastError();
}

}  // namespace isoadv
