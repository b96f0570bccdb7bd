// Device helpers shared by the forward and adjoint kernels of the isoAdvector step (gfx950,
// wave64, FP64): small vectors, the canonical hexahedron's edge tables, a lane's face data, cut
// points, group reductions over the eight lanes of an interface cell, and list appends.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace isoadv {
namespace {

constexpr int kLanes = 8;  // lanes per interface cell

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm3(D3 a) { return sqrt(dot(a, a)); }
// component-wise select (a select of the whole struct can be lowered through memory)
__device__ __forceinline__ D3 sel3(bool c, D3 a, D3 b) { return D3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z}; }

__device__ __forceinline__ bool interface_cell(double a, double eps) { return a > eps && a < 1.0 - eps; }

// Time step of cell c: the scalar one, or its ensemble member's (binary search over the members'
// cell offsets, a table of at most a few hundred bytes that stays in cache).
// the ensemble member holding cell c (0 for a single mesh)
__device__ __forceinline__ int cell_dom(const DevMesh &m, int c) {
    int lo = 0, hi = m.n_dom;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.dom_off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double cell_dt(const DevMesh &m, const double *dt_dom, double dt, int c) {
    return m.n_dom <= 0 ? dt : dt_dom[cell_dom(m, c)];
}

// edges of the canonical hexahedron, and for each face loop position the edge to the next vertex

constexpr bool face_edges_consistent() {
    for (int k = 0; k < 6; ++k)
        for (int i = 0; i < 4; ++i) {
            const int p = kHexFace[k][i], q = kHexFace[k][(i + 1) & 3], e = kFaceEdge[k][i];
            if (!((kEdge[e][0] == p && kEdge[e][1] == q) || (kEdge[e][0] == q && kEdge[e][1] == p))) return false;
        }
    return true;
}
static_assert(face_edges_consistent(), "face/edge tables disagree");


// Work-groups are dispatched to the 8 XCDs round-robin (group b on XCD b mod 8), and each XCD has
// its own L2.  This bijection renumbers groups so that each XCD works through one contiguous
// range (consecutive logical groups, hence neighbouring cells and the faces and stencils they
// share, stay behind one L2).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % kXcds, k = b / kXcds;
    const int q = nb / kXcds, r = nb % kXcds;
    return x * q + min(x, r) + k;
}

// Vertex loop of face lv (lanes 6 and 7 take face 0's) and, as bit i, whether loop position i runs
// along the canonical edge direction.
__device__ __forceinline__ int lane_face_loop(int lv, int *fv) {
    int fwd = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        fv[i] = kHexFace[0][i];
        int e = kFaceEdge[0][i];
#pragma unroll
        for (int k = 1; k < 6; ++k)
            if (lv == k) { fv[i] = kHexFace[k][i]; e = kFaceEdge[k][i]; }
        int first = kEdge[0][0];
#pragma unroll
        for (int t = 1; t < 12; ++t)
            if (e == t) first = kEdge[t][0];
        if (first == fv[i]) fwd |= 1 << i;
    }
    return fwd;
}

// ------------------------------------------------------------------------------------------ faces
// The eight lanes of an interface cell's group split every sub-volume evaluation by face: lane k
// (k < 6) owns canonical face k, its four vertices (relative to the cell's vertex mean), their
// values, and the reciprocal value difference along each of its edges.  Lanes 6 and 7 only help
// gathering vertex values.
struct FaceLane {
    D3 q[4];
    double aq[4];
    double inv[4];  // 1/(a_j - a_i) of the canonical edge (i, j) under loop position k
    int fwd;        // bit k: loop position k runs along the canonical edge direction
    bool planar;
    bool active;
};

// Cut point on the face edge from loop position i to i+1, measured from its wet end; both faces
// sharing the edge evaluate the same expression on the same operands, so they agree bitwise.
__device__ __forceinline__ D3 face_cut(const FaceLane &f, int i, double iso, bool wet_i) {
    const int j = (i + 1) & 3;
    const bool fwd = (f.fwd >> i) & 1;
    const D3 xw = sel3(wet_i, f.q[i], f.q[j]), xd = sel3(wet_i, f.q[j], f.q[i]);
    const double aw = wet_i ? f.aq[i] : f.aq[j];
    // wet end is the canonical edge's first vertex iff (wet_i == fwd)
    const double lam = (wet_i == fwd) ? (iso - aw) * f.inv[i] : (aw - iso) * f.inv[i];
    return xw + lam * (xd - xw);
}

// ------------------------------------------------------------------------------------------ lanes
// Reductions and broadcasts inside a group of 8 consecutive lanes (one interface cell).  The sum
// is a butterfly on DPP lane moves (swap neighbours, swap pairs inside a quad, mirror the two
// quads of the half-row): each step adds the same two partial sums in both partner lanes, so all
// lanes hold bitwise-equal results.  All 8 lanes of a group are active together (every branch
// around a reduction depends only on group-uniform values).
template <int Ctrl>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, Ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), Ctrl, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppSwap1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror: lane i <- lane 7-i within 8
__device__ __forceinline__ double grp_sum(double v) {
    v += dpp_move<kDppSwap1>(v);
    v += dpp_move<kDppSwap2>(v);
    v += dpp_move<kDppHalfMirror>(v);
    return v;
}
__device__ __forceinline__ D3 grp_sum3(D3 v) { return D3{grp_sum(v.x), grp_sum(v.y), grp_sum(v.z)}; }
__device__ __forceinline__ double grp_get(double v, int src) { return __shfl(v, src, 8); }

// Append `count` entries per lane to a device-wide list: one atomic per wave.  Returns the index of
// this lane's first entry.  Every active lane of the wave must call it (count may be 0).
__device__ __forceinline__ int wave_append(int count, int32_t *counter) {
    // the active lanes are a prefix of the wave (a whole wave, or the last wave of a work-group
    // whose size is not a multiple of 64): the highest of them holds the total and takes the slots
    const int lane = __lane_id();
    const int top = 63 - __clzll((unsigned long long)__ballot(1));
    int incl = count;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, top, 64);
    int base = 0;
    if (lane == top && total > 0) base = atomicAdd(counter, total);
    base = __shfl(base, top, 64);
    return base + incl - count;
}

}  // namespace
// ------------------------------------------------------------------------------------------ sweep
// Integral over s in [0, dt] of the submerged fraction of a triangle with signed distances
// d0..d2 from the isoface plane moving with normal speed un: the fraction at time s is
// G(un*s), G the area distribution of d over the triangle (a triangular distribution).
// [0, dt] is split where un*s crosses a vertex distance; on each piece G(un*s) is a quadratic
// in s, integrated exactly by Simpson's rule on the branch picked at the piece's midpoint.
__device__ __forceinline__ double tri_piece(int br, double z, double e1, double e2, double e3, double r31,
                                            double r21, double r32) {
    if (br == 0) return 0.0;
    if (br == 3) return 1.0;
    if (br == 1) {
        const double u = z - e1;
        return (u * r31) * (u * r21);
    }
    const double u = e3 - z;
    return 1.0 - (u * r31) * (u * r32);
}

__device__ __forceinline__ double tri_sweep(double d0, double d1, double d2, double un, double dt) {
    const double e1 = fmin(d0, fmin(d1, d2)), e3 = fmax(d0, fmax(d1, d2));
    const double e2 = fmax(fmin(d0, d1), fmin(fmax(d0, d1), d2));
    const double r31 = e3 > e1 ? 1.0 / (e3 - e1) : 0.0;
    const double r21 = e2 > e1 ? 1.0 / (e2 - e1) : 0.0;
    const double r32 = e3 > e2 ? 1.0 / (e3 - e2) : 0.0;
    auto branch = [&](double z) { return z < e1 ? 0 : (z < e2 ? 1 : (z < e3 ? 2 : 3)); };
    if (un == 0.0) return dt * tri_piece(branch(0.0), 0.0, e1, e2, e3, r31, r21, r32);
    const double inv = 1.0 / un;
    double s1 = e1 * inv, s2 = e2 * inv, s3 = e3 * inv;
    if (un < 0.0) {  // breakpoints in increasing time
        const double t = s1;
        s1 = s3;
        s3 = t;
    }
    const double bk[3] = {s1, s2, s3};
    double I = 0.0, a0 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double a1 = k < 3 ? fmin(fmax(bk[k], 0.0), dt) : dt;
        if (a1 > a0) {
            const double m = 0.5 * (a0 + a1);
            const int br = branch(un * m);
            const double fa = tri_piece(br, un * a0, e1, e2, e3, r31, r21, r32);
            const double fm = tri_piece(br, un * m, e1, e2, e3, r31, r21, r32);
            const double fb = tri_piece(br, un * a1, e1, e2, e3, r31, r21, r32);
            I += (a1 - a0) * (fa + 4.0 * fm + fb) * (1.0 / 6.0);
            a0 = a1;
        }
    }
    return I;
}

}  // namespace isoadv
