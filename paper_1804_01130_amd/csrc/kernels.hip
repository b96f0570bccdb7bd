// HIP kernels of the isoAdvector step for gfx950 (wave64), FP64.
//
// One step (Section 3.2 of the paper) is four launches on one stream:
//   find_surface   interface cells (eps < alpha < 1-eps) compacted by wave ballot + mbcnt
//   surface        per interface cell: vertex values (inverse-distance stencil), isovalue by
//                  bracketing on sorted vertex values + Illinois, isoface centre/normal, and
//                  for every outflow face the time integral of its submerged fraction
//                  (Eqs. tv .. intaplus) -> dV of that face (unique upwind cell: no atomics)
//   update         per cell, gather over its flux faces in ascending face id: dV from the
//                  interface kernel or alpha_upwind*phi*dt (bulk); alpha - sum/V; round-off
//                  chopping; cells beyond the bounds are appended to a list
//   bound          one work-group: Jacobi redistribution over outflow faces of the listed
//                  cells, then chopping (bounding step at the end of Section 3.2)
// Nothing in the step is a dense contraction, so no matrix instructions are used.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace isoadv {
namespace {

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
__device__ __forceinline__ double det3(D3 a, D3 b, D3 c) { return dot(a, cross(b, c)); }

__device__ __forceinline__ bool interface_cell(double a, double eps) { return a > eps && a < 1.0 - eps; }

// edges of the canonical hexahedron and, for each face loop position, the edge to the next vertex
constexpr int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                              {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

// ------------------------------------------------------------------------------------------ cut
// Edge of the canonical hexahedron joining loop positions i and i+1 of face k.
constexpr int kFaceEdge[6][4] = {{3, 2, 1, 0}, {4, 5, 6, 7}, {0, 9, 4, 8}, {1, 10, 5, 9}, {2, 11, 6, 10}, {3, 8, 7, 11}};

constexpr bool face_edges_consistent() {
    for (int k = 0; k < 6; ++k)
        for (int i = 0; i < 4; ++i) {
            const int p = kHexFace[k][i], q = kHexFace[k][(i + 1) & 3], e = kFaceEdge[k][i];
            if (!((kEdge[e][0] == p && kEdge[e][1] == q) || (kEdge[e][0] == q && kEdge[e][1] == p))) return false;
        }
    return true;
}
static_assert(face_edges_consistent(), "face/edge tables disagree");

__device__ __forceinline__ double norm3(D3 a) { return sqrt(dot(a, a)); }

// Cut points of all 12 edges at isovalue iso (meaningful where exactly one end is wet), each
// measured from the wet end so that both faces sharing an edge see the same point.
__device__ __forceinline__ void cut_points(const D3 *X, const double *a, const bool *w, double iso, D3 *cp) {
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        const int i = kEdge[e][0], j = kEdge[e][1];
        const bool wi = w[i];
        const D3 xw = wi ? X[i] : X[j], xd = wi ? X[j] : X[i];
        const double aw = wi ? a[i] : a[j], ad = wi ? a[j] : a[i];
        const double den = ad - aw;
        const double lam = (w[i] != w[j]) ? (iso - aw) / den : 0.0;
        cp[e] = xw + lam * (xd - xw);
    }
}

// Walk the loop of face k: report the wet part's points in order (wet vertices and cut points),
// and every isoface edge on the face as (entry, exit): the wet part leaves the face boundary at
// 'exit' and comes back at 'entry', so the isoface, closing the wet part, runs entry -> exit.
template <class PointFn, class SegFn>
__device__ __forceinline__ void walk_face(int k, const bool *w, const D3 *X, const D3 *cp, PointFn on_point,
                                          SegFn on_seg) {
    D3 exitp{0, 0, 0}, entry0{0, 0, 0};
    bool pending = false, entry_first = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int p = kHexFace[k][i], q = kHexFace[k][(i + 1) & 3], e = kFaceEdge[k][i];
        if (w[p]) on_point(X[p]);
        if (w[p] != w[q]) {
            on_point(cp[e]);
            if (w[p]) {
                exitp = cp[e];
                pending = true;
            } else if (pending) {
                on_seg(cp[e], exitp);
                pending = false;
            } else {
                entry0 = cp[e];
                entry_first = true;
            }
        }
    }
    if (pending && entry_first) on_seg(entry0, exitp);
}

// Six times the wet sub-volume {a > iso} of the cell (local coordinates, origin inside the cell):
// divergence theorem over the wet parts of the faces and the isoface, every polygon fanned about
// its perimeter centroid (length-weighted mean of its edge midpoints), which stays continuous when
// a cut point meets a vertex.  With kIsoface, also twice the isoface area vector (S2) and the sum
// over its fan of (3 x centroid) (x) (2 x area vector) (M, row-major) for the isoface centre.
// tie_wet: a vertex whose value equals iso counts as wet (the limit from below at iso).
template <bool kIsoface>
__device__ __forceinline__ double subvolume6(const D3 *X, const double *a, double iso, bool tie_wet, D3 *S2,
                                             double *M) {
    bool w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = tie_wet ? a[i] >= iso : a[i] > iso;
    D3 cp[12];
    cut_points(X, a, w, iso, cp);
    // isoface apex
    D3 oacc{0, 0, 0}, osum{0, 0, 0};
    double oL = 0.0;
    int nseg = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        walk_face(k, w, X, cp, [](D3) {}, [&](D3 s0, D3 s1) {
            const double l = norm3(s1 - s0);
            oacc = oacc + (0.5 * l) * (s0 + s1);
            oL += l;
            osum = osum + s0;
            ++nseg;
        });
    const D3 o = oL > 0.0 ? (1.0 / oL) * oacc : (nseg > 0 ? (1.0 / nseg) * osum : D3{0, 0, 0});
    if (kIsoface) {
        *S2 = D3{0, 0, 0};
#pragma unroll
        for (int q = 0; q < 9; ++q) M[q] = 0.0;
    }
    double v6 = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        // perimeter centroid of the wet part of the face
        D3 first{0, 0, 0}, prev{0, 0, 0}, pacc{0, 0, 0}, psum{0, 0, 0};
        double pl = 0.0;
        int cnt = 0;
        walk_face(k, w, X, cp, [&](D3 x) {
            if (cnt > 0) {
                const double l = norm3(x - prev);
                pacc = pacc + (0.5 * l) * (x + prev);
                pl += l;
            } else {
                first = x;
            }
            prev = x;
            psum = psum + x;
            ++cnt;
        }, [](D3, D3) {});
        if (cnt > 0) {
            const double l = norm3(first - prev);
            pacc = pacc + (0.5 * l) * (first + prev);
            pl += l;
        }
        const D3 ap = pl > 0.0 ? (1.0 / pl) * pacc : (cnt > 0 ? (1.0 / cnt) * psum : D3{0, 0, 0});
        // fan of the wet part, isoface triangles on this face
        D3 f2{0, 0, 0}, p2{0, 0, 0};
        int c2 = 0;
        walk_face(k, w, X, cp, [&](D3 x) {
            if (c2 > 0) v6 += det3(ap, p2, x); else f2 = x;
            p2 = x;
            ++c2;
        }, [&](D3 s0, D3 s1) {
            v6 += det3(o, s0, s1);
            if (kIsoface) {
                const D3 t = cross(s0 - o, s1 - o);
                *S2 = *S2 + t;
                const D3 g = o + s0 + s1;
                M[0] += g.x * t.x; M[1] += g.x * t.y; M[2] += g.x * t.z;
                M[3] += g.y * t.x; M[4] += g.y * t.y; M[5] += g.y * t.z;
                M[6] += g.z * t.x; M[7] += g.z * t.y; M[8] += g.z * t.z;
            }
        });
        if (c2 >= 3) v6 += det3(ap, p2, f2);
    }
    return v6;
}

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
        double u = z - e1;
        return (u * r31) * (u * r21);
    }
    double u = e3 - z;
    return 1.0 - (u * r31) * (u * r32);
}

__device__ __forceinline__ double tri_sweep(double d0, double d1, double d2, double un, double dt) {
    // sort ascending (median of three by min/max)
    const double e1 = fmin(d0, fmin(d1, d2)), e3 = fmax(d0, fmax(d1, d2));
    const double e2 = fmax(fmin(d0, d1), fmin(fmax(d0, d1), d2));
    double r31 = e3 > e1 ? 1.0 / (e3 - e1) : 0.0;
    double r21 = e2 > e1 ? 1.0 / (e2 - e1) : 0.0;
    double r32 = e3 > e2 ? 1.0 / (e3 - e2) : 0.0;
    auto branch = [&](double z) { return z < e1 ? 0 : (z < e2 ? 1 : (z < e3 ? 2 : 3)); };
    if (un == 0.0) return dt * tri_piece(branch(0.0), 0.0, e1, e2, e3, r31, r21, r32);
    // breakpoints in (0, dt)
    double b[3];
    int nb = 0;
    double inv = 1.0 / un;
    double s1 = e1 * inv, s2 = e2 * inv, s3 = e3 * inv;
    if (s1 > 0.0 && s1 < dt) b[nb++] = s1;
    if (s2 > 0.0 && s2 < dt) b[nb++] = s2;
    if (s3 > 0.0 && s3 < dt) b[nb++] = s3;
    if (un < 0.0) {  // breakpoints come in decreasing order
        double t = b[0];
        if (nb == 2) { b[0] = b[1]; b[1] = t; }
        if (nb == 3) { b[0] = b[2]; b[2] = t; }
    }
    double I = 0.0, a0 = 0.0;
    for (int k = 0; k <= nb; ++k) {
        double a1 = k < nb ? b[k] : dt;
        if (a1 > a0) {
            double m = 0.5 * (a0 + a1);
            int br = branch(un * m);
            double fa = tri_piece(br, un * a0, e1, e2, e3, r31, r21, r32);
            double fm = tri_piece(br, un * m, e1, e2, e3, r31, r21, r32);
            double fb = tri_piece(br, un * a1, e1, e2, e3, r31, r21, r32);
            I += (a1 - a0) * (fa + 4.0 * fm + fb) * (1.0 / 6.0);
        }
        a0 = a1;
    }
    return I;
}

// ------------------------------------------------------------------------------------------ kernels
__global__ void __launch_bounds__(1024) k_find_surface(const double *__restrict__ alpha, int n, double eps,
                                                       int32_t *__restrict__ list, int32_t cap,
                                                       int32_t *__restrict__ counters, int32_t *__restrict__ kind) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool s = false;
    if (c < n) {
        s = interface_cell(alpha[c], eps);
        if (kind) kind[c] = 0;
    }
    uint64_t mask = __ballot(s);
    if (mask == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[kCntSurf], __popcll(mask));
    base = __shfl(base, leader);
    if (s) {
        int pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (pos < cap) list[pos] = c;
        else atomicAdd(&counters[kCntOverflow], 1);
    }
}

struct SurfArgs {
    DevMesh m;
    const double *alpha, *phi, *U;
    double dt, eps, flat_tol;
    int32_t max_iter;
    const int32_t *list;
    const int32_t *counters;
    int32_t cap;
    double *dvs;
    int32_t *cnt_out;
    int want_stats;
    iso_trace tr;
};

__global__ void __launch_bounds__(256) k_surface(SurfArgs A) {
    int n = min(A.counters[kCntSurf], A.cap);
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int iters = 0, flat = 0, nonconv = 0;
    for (; idx < n; idx += gridDim.x * blockDim.x) {
        const int c = A.list[idx];
        const DevMesh &m = A.m;
        const double aP = A.alpha[c];
        const double V = m.vol[c];
        // vertex coordinates relative to the vertex mean
        D3 X[8];
        const double *cx = m.cxyz + 24 * (size_t)c;
#pragma unroll
        for (int i = 0; i < 8; ++i) X[i] = D3{cx[3 * i], cx[3 * i + 1], cx[3 * i + 2]};
        D3 xm{0, 0, 0};
#pragma unroll
        for (int i = 0; i < 8; ++i) xm = xm + X[i];
        xm = 0.125 * xm;
#pragma unroll
        for (int i = 0; i < 8; ++i) X[i] = X[i] - xm;
        // vertex values: normalised inverse-distance stencils of the point classes
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int k = m.cpt[8 * (size_t)c + i];
            int e0 = m.st_ptr[k], e1 = m.st_ptr[k + 1];
            double s = 0.0;
            for (int e = e0; e < e1; ++e) s += m.st_w[e] * A.alpha[m.st_cell[e]];
            a[i] = s;
        }
        if (A.tr.vert_alpha) {
#pragma unroll
            for (int i = 0; i < 8; ++i) A.tr.vert_alpha[8 * (size_t)c + i] = a[i];
        }
        double lo = a[0], hi = a[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) { lo = fmin(lo, a[i]); hi = fmax(hi, a[i]); }

        bool recon = hi - lo > A.flat_tol;
        double iso = 0.0;
        int it = 0;
        D3 nS{0, 0, 0}, xS{0, 0, 0};
        double un = 0.0;
        if (recon) {
            // sorted vertex values (insertion sort, 8 elements)
            double s[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) s[i] = a[i];
#pragma unroll
            for (int i = 1; i < 8; ++i)
#pragma unroll
                for (int j = i; j > 0; --j) {
                    double x = fmin(s[j - 1], s[j]), y = fmax(s[j - 1], s[j]);
                    s[j - 1] = x;
                    s[j] = y;
                }
            const double V6 = 6.0 * V;
            auto f = [&](double x, bool tie_wet) {
                return subvolume6<false>(X, a, x, tie_wet, nullptr, nullptr) / V6 - aP;
            };
            // bracket between consecutive sorted vertex values: V_sub is a cubic there
            int il = 0, ih = 7;
            double fl = 1.0 - aP, fh = -aP;
            bool exact = false;
            auto sorted_at = [&](int i) {  // s[i] without dynamic register indexing
                double r = s[0];
#pragma unroll
                for (int q = 1; q < 8; ++q) r = i == q ? s[q] : r;
                return r;
            };
            while (ih - il > 1) {
                int im = (il + ih) >> 1;
                double sm = sorted_at(im);
                double fm = f(sm, false);
                ++it;
                if (fm > 0.0) { il = im; fl = fm; }
                else if (fm < 0.0) { ih = im; fh = fm; }
                else { iso = sm; exact = true; break; }
            }
            if (!exact) {
                // Between consecutive vertex values the sub-volume is smooth; at a vertex value it may
                // jump.  If it jumps across alpha_P at the upper bracket, that value is the isovalue.
                double x0 = sorted_at(il), x1 = sorted_at(ih), f0 = fl;
                double f1 = f(x1, true);  // limit from below at x1
                ++it;
                if (f1 > 0.0) {
                    iso = x1;
                } else {
                    // Illinois (modified regula falsi) with a bisection guard, to round-off
                    int side = 0;
                    bool conv = false;
                    for (; it < A.max_iter; ++it) {
                        double wdt = x1 - x0;
                        if (!(wdt > 4.0 * __DBL_EPSILON__ * fmax(fabs(x0), fabs(x1)))) { conv = true; break; }
                        double x = x1 - f1 * (x1 - x0) / (f1 - f0);
                        if (!(x > x0 && x < x1) || (it & 7) == 7) x = x0 + 0.5 * wdt;
                        double fx = f(x, false);
                        if (fx == 0.0 || fabs(fx) <= 4.0 * __DBL_EPSILON__) {
                            x0 = x1 = x;
                            f0 = f1 = fx;
                            conv = true;
                            ++it;
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
            // isoface at the isovalue
            D3 S2;
            double M[9];
            subvolume6<true>(X, a, iso, false, &S2, M);
            double nrm = sqrt(dot(S2, S2));
            if (nrm > 0.0) {
                nS = (1.0 / nrm) * S2;
                double wsum = dot(S2, nS);  // sum of 2*area projections
                // x_S = sum_t (S_t . n) g_t / sum_t (S_t . n), with g_t = (sum of 3 points)/3
                D3 num{M[0] * nS.x + M[1] * nS.y + M[2] * nS.z, M[3] * nS.x + M[4] * nS.y + M[5] * nS.z,
                       M[6] * nS.x + M[7] * nS.y + M[8] * nS.z};
                xS = (1.0 / (3.0 * wsum)) * num;
                un = A.U[c] * nS.x + A.U[m.n_cells + c] * nS.y + A.U[2 * (size_t)m.n_cells + c] * nS.z;
            } else {
                recon = false;
            }
        }
        if (!recon) ++flat;
        if (A.tr.kind) A.tr.kind[c] = recon ? 1 : 2;
        if (recon) {
            if (A.tr.iso) A.tr.iso[c] = iso;
            if (A.tr.iters) A.tr.iters[c] = it;
            if (A.tr.rec) {
                double *r = A.tr.rec + 7 * (size_t)c;
                r[0] = xS.x + xm.x; r[1] = xS.y + xm.y; r[2] = xS.z + xm.z;
                r[3] = nS.x; r[4] = nS.y; r[5] = nS.z; r[6] = un;
            }
        }
        iters = max(iters, it);
        // outflow faces of this cell: dV = phi * time-integrated submerged fraction
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            int32_t v = m.lface[6 * (size_t)c + k];
            if (v == kEmpty) continue;
            int32_t fid = v >= 0 ? v : ~v;
            double ph = A.phi[fid];
            double out = v >= 0 ? ph : -ph;
            if (!(out > 0.0)) continue;
            double dv;
            if (recon) {
                D3 q[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) q[i] = X[kHexFace[k][i]];
                D3 ap = 0.25 * (q[0] + q[1] + q[2] + q[3]);
                double dap = dot(ap - xS, nS);
                double dq[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) dq[i] = dot(q[i] - xS, nS);
                double acc = 0.0, Af = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    D3 cr = cross(q[i] - ap, q[(i + 1) & 3] - ap);
                    double Ai = 0.5 * sqrt(dot(cr, cr));
                    acc += Ai * tri_sweep(dap, dq[i], dq[(i + 1) & 3], un, A.dt);
                    Af += Ai;
                }
                dv = ph * (acc / Af);
            } else {
                dv = aP * ph * A.dt;
            }
            A.dvs[fid] = dv;
        }
    }
    if (A.want_stats) {
        // wave reductions, then one atomic per wave
        for (int off = 32; off > 0; off >>= 1) {
            iters = max(iters, __shfl_xor(iters, off));
            flat += __shfl_xor(flat, off);
            nonconv += __shfl_xor(nonconv, off);
        }
        if (__lane_id() == 0) {
            if (iters) atomicMax(&A.cnt_out[kCntMaxIter], iters);
            if (flat) atomicAdd(&A.cnt_out[kCntFlat], flat);
            if (nonconv) atomicAdd(&A.cnt_out[kCntNonconv], nonconv);
        }
    }
}

struct UpdArgs {
    DevMesh m;
    const double *alpha, *phi, *dvs;
    double dt, eps, tol;
    int clip;
    double *alpha_new;
    int32_t *olist;
    int32_t *counters;
    double *trace_dV, *trace_raw;
};

__global__ void __launch_bounds__(1024) k_update(UpdArgs A) {
    const int n = A.m.n_cells;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool offend = false;
    if (c < n) {
        const double aP = A.alpha[c];
        const bool sP = interface_cell(aP, A.eps);
        double sum = 0.0;
        for (int k = 0; k < A.m.W; ++k) {
            int32_t v = A.m.slot_face[(size_t)k * n + c];
            if (v == kEmpty) break;
            int32_t fid = v >= 0 ? v : ~v;
            double ph = A.phi[fid];
            double out = v >= 0 ? ph : -ph;
            double dv = 0.0;
            if (out > 0.0) {
                dv = sP ? A.dvs[fid] : aP * ph * A.dt;
            } else if (out < 0.0) {
                int32_t o = A.m.slot_nbr[(size_t)k * n + c];
                if (o >= 0) {
                    double ao = A.alpha[o];
                    dv = interface_cell(ao, A.eps) ? A.dvs[fid] : ao * ph * A.dt;
                } else {
                    dv = A.m.patch_alpha[-1 - o] * ph * A.dt;
                }
            }
            sum += v >= 0 ? dv : -dv;
            if (A.trace_dV && v >= 0) A.trace_dV[fid] = dv;
        }
        double x = aP - sum / A.m.vol[c];
        if (A.trace_raw) A.trace_raw[c] = x;
        if (A.clip) {
            if (x < 0.0 && x >= -A.tol) x = 0.0;
            else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
        }
        offend = x > 1.0 + A.tol || x < -A.tol;
        A.alpha_new[c] = x;
    }
    uint64_t mask = __ballot(offend);
    if (mask == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&A.counters[kCntOff], __popcll(mask));
    base = __shfl(base, leader);
    if (offend)
        A.olist[base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))] = c;
}

struct BoundArgs {
    DevMesh m;
    const double *alpha, *phi, *dvs;
    double dt, eps, tol;
    int clip, n_iter;
    double *alpha_new;
    DevWork w;
};

// Current dV of outflow face fid of cell P (P is its upwind cell).
__device__ __forceinline__ double face_dv_now(const BoundArgs &A, int32_t fid, bool sP, double aold, double ph) {
    if (A.w.fmark[fid]) return A.w.dvcur[fid];
    return sP ? A.dvs[fid] : aold * ph * A.dt;
}

__device__ __forceinline__ void claim(BoundArgs &A, int32_t q, int *nT) {
    if (atomicExch(&A.w.cmark[q], 1) == 0) {
        int pos = atomicAdd(nT, 1);
        A.w.tlist[pos] = q;
    }
}

__global__ void __launch_bounds__(1024) k_bound(BoundArgs A) {
    __shared__ int nO, nT, nF, nNext;
    const int n = A.m.n_cells;
    const int tid = threadIdx.x, nt = blockDim.x;
    int32_t *cur = A.w.olist, *nxt = A.w.olist + n;
    if (tid == 0) {
        nO = A.w.counters[kCntOff];
        nF = 0;
    }
    __syncthreads();
    for (int it = 0; it < A.n_iter; ++it) {
        if (nO == 0) break;
        if (tid == 0) { nT = 0; nNext = 0; }
        __syncthreads();
        // A: corrections on the outflow faces of the listed cells
        for (int i = tid; i < nO; i += nt) {
            const int32_t P = cur[i];
            const double a = A.alpha_new[P];
            const bool over = a > 1.0 + A.tol;
            const double aold = A.alpha[P];
            const bool sP = interface_cell(aold, A.eps);
            double sumcap = 0.0;
            for (int k = 0; k < A.m.W; ++k) {
                int32_t v = A.m.slot_face[(size_t)k * n + P];
                if (v == kEmpty) break;
                int32_t fid = v >= 0 ? v : ~v;
                double ph = A.phi[fid];
                double outphi = v >= 0 ? ph : -ph;
                if (!(outphi > 0.0)) continue;
                double dv = face_dv_now(A, fid, sP, aold, ph);
                double outv = v >= 0 ? dv : -dv;
                double cap = over ? outphi * A.dt - outv : outv;
                if (cap > 0.0) sumcap += cap;
            }
            claim(A, P, &nT);
            if (!(sumcap > 0.0)) continue;
            double need = over ? (a - 1.0) * A.m.vol[P] : -a * A.m.vol[P];
            double r = fmin(need / sumcap, 1.0);
            for (int k = 0; k < A.m.W; ++k) {
                int32_t v = A.m.slot_face[(size_t)k * n + P];
                if (v == kEmpty) break;
                int32_t fid = v >= 0 ? v : ~v;
                double ph = A.phi[fid];
                double outphi = v >= 0 ? ph : -ph;
                if (!(outphi > 0.0)) continue;
                double dv = face_dv_now(A, fid, sP, aold, ph);
                double outv = v >= 0 ? dv : -dv;
                double cap = over ? outphi * A.dt - outv : outv;
                if (!(cap > 0.0)) continue;
                double d = cap * r;
                A.w.delta[fid] = over ? (v >= 0 ? d : -d) : (v >= 0 ? -d : d);
                int32_t q = A.m.slot_nbr[(size_t)k * n + P];
                if (q >= 0) claim(A, q, &nT);
            }
        }
        __syncthreads();
        // B: apply to every touched cell, fixed face order
        const bool last = it == A.n_iter - 1;
        for (int i = tid; i < nT; i += nt) {
            const int32_t Q = A.w.tlist[i];
            double sum = 0.0;
            for (int k = 0; k < A.m.W; ++k) {
                int32_t v = A.m.slot_face[(size_t)k * n + Q];
                if (v == kEmpty) break;
                int32_t fid = v >= 0 ? v : ~v;
                double d = A.w.delta[fid];
                sum += v >= 0 ? d : -d;
            }
            double x = A.alpha_new[Q] - sum / A.m.vol[Q];
            if (A.clip) {
                if (x < 0.0 && x >= -A.tol) x = 0.0;
                else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
                if (last) x = fmin(fmax(x, 0.0), 1.0);
            }
            A.alpha_new[Q] = x;
            A.w.cmark[Q] = 0;
            if (x > 1.0 + A.tol || x < -A.tol) nxt[atomicAdd(&nNext, 1)] = Q;
        }
        __syncthreads();
        // C: commit the face changes, clear the corrections
        for (int i = tid; i < nO; i += nt) {
            const int32_t P = cur[i];
            const double aold = A.alpha[P];
            const bool sP = interface_cell(aold, A.eps);
            for (int k = 0; k < A.m.W; ++k) {
                int32_t v = A.m.slot_face[(size_t)k * n + P];
                if (v == kEmpty) break;
                int32_t fid = v >= 0 ? v : ~v;
                double ph = A.phi[fid];
                double outphi = v >= 0 ? ph : -ph;
                if (!(outphi > 0.0)) continue;
                double dv = face_dv_now(A, fid, sP, aold, ph);
                A.w.dvcur[fid] = dv + A.w.delta[fid];
                A.w.delta[fid] = 0.0;
                if (A.w.fmark[fid] == 0) {
                    A.w.fmark[fid] = 1;
                    A.w.flist[atomicAdd(&nF, 1)] = fid;
                }
            }
        }
        __syncthreads();
        int32_t *t = cur; cur = nxt; nxt = t;
        if (tid == 0) nO = nNext;
        __syncthreads();
    }
    if (A.n_iter == 0 && A.clip) {
        for (int i = tid; i < nO; i += nt) {
            int32_t P = cur[i];
            A.alpha_new[P] = fmin(fmax(A.alpha_new[P], 0.0), 1.0);
        }
    }
    __syncthreads();
    for (int i = tid; i < nF; i += nt) A.w.fmark[A.w.flist[i]] = 0;
    __syncthreads();
    // keep this step's counters for the statistics, zero them for the next step
    if (tid < 8) {
        int32_t x = A.w.counters[tid];
        A.w.counters[8 + tid] = tid == kCntActive0 ? A.w.counters[kCntOff] : x;
    }
    __syncthreads();
    if (tid < 8) A.w.counters[tid] = 0;
}

__global__ void __launch_bounds__(1024) k_stats(const double *alpha, const double *alpha_new, const double *vol, int n,
                                                double *red) {
    __shared__ double sb[1024], sa[1024], smin[1024], smax[1024];
    double b = 0, a = 0, mn = 1e300, mx = -1e300;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        b += alpha[c] * vol[c];
        a += alpha_new[c] * vol[c];
        mn = fmin(mn, alpha_new[c]);
        mx = fmax(mx, alpha_new[c]);
    }
    int t = threadIdx.x;
    sb[t] = b; sa[t] = a; smin[t] = mn; smax[t] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
            sb[t] += sb[t + s]; sa[t] += sa[t + s];
            smin[t] = fmin(smin[t], smin[t + s]); smax[t] = fmax(smax[t], smax[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) { red[0] = sb[0]; red[1] = sa[0]; red[2] = smin[0]; red[3] = smax[0]; red[4] = 0.0; }
}

}  // namespace

hipError_t launch_step(const DevMesh &m, const DevWork &w, const Params &p, const StepArgs &a, const iso_trace *trace,
                       int block_cells, int block_surface, bool want_stats, hipStream_t s, hipEvent_t *ev) {
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    const int n = m.n_cells;
    iso_trace tr{};
    if (trace) tr = *trace;
    int gc = (n + block_cells - 1) / block_cells;
    mark(0);
    hipLaunchKernelGGL(k_find_surface, dim3(gc), dim3(block_cells), 0, s, a.alpha, n, p.eps_surf, w.surf, w.cap,
                       w.counters, tr.kind);
    SurfArgs sa{m, a.alpha, a.phi, a.U, a.dt, p.eps_surf, p.flat_tol, p.root_max_iter, w.surf, w.counters, w.cap,
                w.dvs, w.counters, want_stats ? 1 : 0, tr};
    int gs_max = (w.cap + block_surface - 1) / block_surface;
    int gs = std::min(gs_max, 2048 * 64 / block_surface);
    gs = std::max(gs, 1);
    mark(1);
    hipLaunchKernelGGL(k_surface, dim3(gs), dim3(block_surface), 0, s, sa);
    mark(2);
    UpdArgs ua{m, a.alpha, a.phi, w.dvs, a.dt, p.eps_surf, p.bound_tol, p.clip, a.alpha_new, w.olist, w.counters,
               tr.dV, tr.alpha_raw};
    hipLaunchKernelGGL(k_update, dim3(gc), dim3(block_cells), 0, s, ua);
    mark(3);
    BoundArgs ba{m, a.alpha, a.phi, w.dvs, a.dt, p.eps_surf, p.bound_tol, p.clip, p.n_bound_iter, a.alpha_new, w};
    hipLaunchKernelGGL(k_bound, dim3(1), dim3(1024), 0, s, ba);
    mark(4);
    return hipGetLastError();
}

hipError_t launch_stats(const DevMesh &m, const DevWork &w, const double *alpha, const double *alpha_new,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, s, alpha, alpha_new, m.vol, m.n_cells, w.red);
    return hipGetLastError();
}

}  // namespace isoadv
