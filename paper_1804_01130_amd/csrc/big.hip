// Interface cells of general polyhedra (Section 3: arbitrary polyhedral control volumes; Section
// 3.2: the isoface construction on them): cells beyond what the eight-lane kernel takes (more
// than six faces, more than eight points, or faces of more than four points), up to kBigPts
// points, kBigFaces faces and kBigFacePts points per face.
//
// Sixteen lanes per cell, one per face (the eight-lane kernel skips these cells).  The cell's
// points, relative to their mean, and their vertex values sit in LDS, where every lane of the
// group reads them; each lane keeps its face's loop of local point indices in registers, and,
// when no face has more than four points, the face's points themselves and the reciprocal value
// difference of each edge (the kFP = 4 instantiation: no LDS reads and no divisions in the
// isovalue search).  The construction is the eight-lane kernel's generic path:
//   vertex values through the inverse-distance stencils (two points per lane); the sorted values
//   by rank; the isovalue bracketed between two consecutive sorted values (the limit from above
//   at each), then found by Newton on the bracket's functional form when every face is planar,
//   by Illinois with a bisection guard otherwise, to round-off, or taken at a vertex value where
//   the sub-volume jumps; the sub-volume by the divergence theorem, each lane's wet loop
//   fanned about a face point (planar faces) or its perimeter centroid, the isoface fanned about
//   the perimeter centroid of its edges; the isoface's normal, centre and U_P . n_S; and each
//   lane's swept integral of its face, over the triangles that fan it about its vertex mean.
// Face sums are reduced over the sixteen lanes by a butterfly in which partner lanes add the same
// two partial sums, so every lane holds bitwise the same totals and takes the same branches of
// the root search.
#include "device_common.h"
#include "internal.h"

namespace isoadv {

namespace {

constexpr int kGrp = 16;         // lanes per cell, one per face
constexpr int kGrpPerBlock = 16; // 256 threads
static_assert(kBigFaces == kGrp, "one lane per face");
static_assert(kBigPts == 2 * kGrp, "two points per lane");
static_assert(kBigFacePts <= 16, "a face loop packs into four words of bytes");

struct Pt {
    double x, y, z, a;  // point relative to the cell's point mean, and its vertex value
};

// This lane's face: its loop of local point indices (byte i of the four words: position i); for
// faces of at most four points (kFP = 4) also the points and, for edge i (position i to i + 1),
// 1 / (a_low - a_high) of its two vertex values (0 when they are equal).
template <int kFP>
struct FaceLoop {
    int n;  // points; 0 when the lane has no face
    int planar;
    uint32_t w[4];
    Pt q[kFP <= 4 ? kFP : 1];
    double r[kFP <= 4 ? kFP : 1];
};

template <int kFP>
__device__ __forceinline__ int loop_at(const FaceLoop<kFP> &L, int i) { return (L.w[i >> 2] >> (8 * (i & 3))) & 0xff; }

template <int kFP>
__device__ __forceinline__ Pt fetch(const Pt *P, const FaceLoop<kFP> &L, int i) {
    if constexpr (kFP <= 4) return L.q[i];
    else return P[loop_at(L, i)];
}

// Sum over the sixteen lanes of a group: the eight-lane butterfly, then the two halves of the row
// swapped by mirroring (lane i <- lane 15 - i).
constexpr int kDppRowMirror = 0x140;
__device__ __forceinline__ double g16(double v) {
    v = grp_sum(v);
    return v + dpp_move<kDppRowMirror>(v);
}
__device__ __forceinline__ D3 g16_3(D3 v) { return D3{g16(v.x), g16(v.y), g16(v.z)}; }

// Order the group's LDS writes before the reads of other lanes of the same wave.
__device__ __forceinline__ void grp_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ D3 xyz(const Pt &p) { return D3{p.x, p.y, p.z}; }

// Cut point on the edge between two points of which exactly one is wet: from the wet end, so that
// the two faces sharing the edge compute the same point.
__device__ __forceinline__ D3 edge_cut(const Pt &w, const Pt &d, double iso) {
    const double lam = (iso - w.a) / (d.a - w.a);
    return xyz(w) + lam * (xyz(d) - xyz(w));
}

// Cut point on edge i, from point pi to point pj, exactly one of them wet: from the wet end (the
// one of higher value).
template <int kFP>
__device__ __forceinline__ D3 cut_at(const FaceLoop<kFP> &L, int i, const Pt &pi, const Pt &pj, bool wi, double iso) {
    const Pt w = wi ? pi : pj, d = wi ? pj : pi;
    if constexpr (kFP <= 4) return xyz(w) + ((iso - w.a) * L.r[i]) * (xyz(d) - xyz(w));
    else return edge_cut(w, d, iso);
}

struct FacePart {
    double v6;
    D3 cseg, oacc;
    double oL;
};

// s0 x s1 rounded without contraction, so that s1 x s0 is its exact negative: when the wet part
// around a point with only two edges in the cell is a sliver, the two faces at the point add
// opposite isoface edges, which then cancel to an exact zero area (no isoface, a flat cell).
__device__ __forceinline__ D3 cross_antisym(D3 a, D3 b) {
#pragma clang fp contract(off)
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ void iso_edge(FacePart &r, D3 s0, D3 s1) {
    const double l = norm3(s1 - s0);
    r.cseg = r.cseg + cross_antisym(s0, s1);
    r.oacc = r.oacc + (0.5 * l) * (s0 + s1);
    r.oL += l;
}

// This lane's face share of six times the wet sub-volume and of the isoface sums.  An entry into
// the wet part closes the isoface edge from the preceding exit; an entry before the loop's first
// exit pairs with its last one.
template <int kFP>
__device__ FacePart face_part(const Pt *P, const FaceLoop<kFP> &L, double iso, bool tie_wet) {
    FacePart r{0.0, {0, 0, 0}, {0, 0, 0}, 0.0};
    if (L.n == 0) return r;
    D3 C{0, 0, 0}, pacc{0, 0, 0}, psum{0, 0, 0}, lastexit{0, 0, 0}, first_entry{0, 0, 0};
    double pl = 0.0;
    int cnt = 0;
    bool have_exit = false, pend = false;
    const Pt p0 = fetch(P, L, 0);
    Pt pi = p0;
    bool wi = tie_wet ? p0.a >= iso : p0.a > iso;
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
        if (i < L.n) {
            Pt pj = p0;
            if (i + 1 < kFP && i + 1 < L.n) pj = fetch(P, L, i + 1);
            const bool wj = tie_wet ? pj.a >= iso : pj.a > iso;
            const D3 xi = xyz(pi), xj = xyz(pj);
            D3 cut{0, 0, 0};
            if (wi != wj) cut = cut_at(L, i, pi, pj, wi, iso);
            if (!wi && wj) {
                if (have_exit) iso_edge(r, cut, lastexit);
                else { pend = true; first_entry = cut; }
            }
            if (wi && !wj) { lastexit = cut; have_exit = true; }
            if (wi || wj) {
                const D3 u = wi ? xi : cut, v = wj ? xj : cut;
                C = C + cross(u, v);
                const double l = norm3(v - u);
                pacc = pacc + (0.5 * l) * (u + v);
                pl += l;
            }
            if (wi) psum = psum + xi;
            if (wi != wj) psum = psum + cut;
            cnt += (wi ? 1 : 0) + (wi != wj ? 1 : 0);
            pi = pj;
            wi = wj;
        }
    }
    if (pend) iso_edge(r, first_entry, lastexit);
    C = C - r.cseg;  // the isoface edges close the wet loop, walked exit to entry
    if (cnt >= 3) {
        D3 ap = xyz(p0);
        if (!L.planar) {
            const D3 tot = pacc + r.oacc;
            const double tl = pl + r.oL;
            ap = tl > 0.0 ? (1.0 / tl) * tot : (1.0 / cnt) * psum;
        }
        r.v6 = dot(ap, C);
    }
    return r;
}

// Six times the wet sub-volume of the cell at isovalue iso (every lane of the group calls it and
// gets the same result), with the isoface's fan apex and area-vector sum.
template <int kFP>
__device__ __forceinline__ double grp_vsub6(const Pt *P, const FaceLoop<kFP> &L, double iso, bool tie_wet, D3 &o,
                                            D3 &cseg) {
    const FacePart r = face_part(P, L, iso, tie_wet);
    const double v6 = g16(r.v6), oL = g16(r.oL);
    cseg = g16_3(r.cseg);
    const D3 oacc = g16_3(r.oacc);
    o = oL > 0.0 ? (1.0 / oL) * oacc : D3{0, 0, 0};
    return v6 + dot(o, cseg);
}

// Inside a bracket (xr, xr + uhi) between consecutive vertex values the wet pattern is fixed
// (wet: a > xr) and every cut point moves linearly with u = iso - xr.  On a planar face the
// lane's share of six times the sub-volume is ap . C(u), a quadratic, and the isoface adds
// o(u) . B(u) with B the sum of its edges' s x e; the lane returns its share of the value and
// of the derivative in u of each sum, for Newton's method on the group totals.
struct IntervalPart {
    double v, dv;      // ap . C(u) and its derivative
    D3 B, dB;          // this face's isoface edges: sum s x e, and its derivative
    D3 oacc, doacc;    // their length x midpoint, and its derivative
    double oL, doL;    // their length, and its derivative
};

template <int kFP>
__device__ IntervalPart face_interval(const Pt *P, const FaceLoop<kFP> &L, double xr, double u) {
    IntervalPart r{0.0, 0.0, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}, 0.0, 0.0};
    if (L.n == 0) return r;
    const double iso = xr + u;
    const D3 Z{0, 0, 0};
    D3 C = Z, dC = Z, le0 = Z, le1 = Z, fe0 = Z, fe1 = Z;
    int cnt = 0;
    bool have_exit = false, pend = false;
    auto seg = [&](D3 s0, D3 s1, D3 e0, D3 e1) {
        const D3 d = e0 - s0, dd = e1 - s1;
        const double l = norm3(d);
        const double dl = l > 0.0 ? dot(d, dd) / l : 0.0;
        r.B = r.B + cross_antisym(s0, e0);
        r.dB = r.dB + cross(s1, e0) + cross(s0, e1);
        r.oacc = r.oacc + (0.5 * l) * (s0 + e0);
        r.doacc = r.doacc + (0.5 * dl) * (s0 + e0) + (0.5 * l) * (s1 + e1);
        r.oL += l;
        r.doL += dl;
    };
    const Pt p0 = fetch(P, L, 0);
    Pt pi = p0;
    bool wi = p0.a > xr;
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
        if (i < L.n) {
            Pt pj = p0;
            if (i + 1 < kFP && i + 1 < L.n) pj = fetch(P, L, i + 1);
            const bool wj = pj.a > xr;
            const D3 xi = xyz(pi), xj = xyz(pj);
            D3 c0 = Z, c1 = Z;
            if (wi != wj) {
                const Pt w = wi ? pi : pj, d = wi ? pj : pi;
                double rr;
                if constexpr (kFP <= 4) rr = L.r[i];
                else rr = 1.0 / (d.a - w.a);
                c0 = xyz(w) + ((iso - w.a) * rr) * (xyz(d) - xyz(w));
                c1 = rr * (xyz(d) - xyz(w));
            }
            if (!wi && wj) {
                if (have_exit) seg(c0, c1, le0, le1);
                else { pend = true; fe0 = c0; fe1 = c1; }
            }
            if (wi && !wj) { le0 = c0; le1 = c1; have_exit = true; }
            if (wi || wj) {
                const D3 U0 = wi ? xi : c0, U1 = wi ? Z : c1, V0 = wj ? xj : c0, V1 = wj ? Z : c1;
                C = C + cross(U0, V0);
                dC = dC + cross(U1, V0) + cross(U0, V1);
            }
            cnt += (wi ? 1 : 0) + (wi != wj ? 1 : 0);
            pi = pj;
            wi = wj;
        }
    }
    if (pend) seg(fe0, fe1, le0, le1);
    if (cnt >= 3) {
        const D3 ap = xyz(p0);
        r.v = dot(ap, C - r.B);
        r.dv = dot(ap, dC - r.dB);
    }
    return r;
}

// This lane's share of the isoface centroid: the fan triangles (o, entry, preceding exit) of its
// face's isoface edges, weighted by their area along n_S.
template <int kFP>
__device__ void face_centre(const Pt *P, const FaceLoop<kFP> &L, double iso, D3 o, D3 nS, D3 &acc, double &ws) {
    acc = D3{0, 0, 0};
    ws = 0.0;
    if (L.n == 0) return;
    D3 lastexit{0, 0, 0}, first_entry{0, 0, 0};
    bool have_exit = false, pend = false;
    const Pt p0 = fetch(P, L, 0);
    Pt pi = p0;
    bool wi = p0.a > iso;
    auto tri = [&](D3 s0, D3 s1) {
        const double wt = dot(cross(s0 - o, s1 - o), nS);
        acc = acc + wt * (o + s0 + s1);
        ws += wt;
    };
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
        if (i < L.n) {
            Pt pj = p0;
            if (i + 1 < kFP && i + 1 < L.n) pj = fetch(P, L, i + 1);
            const bool wj = pj.a > iso;
            if (!wi && wj) {
                const D3 cut = cut_at(L, i, pi, pj, false, iso);
                if (have_exit) tri(cut, lastexit);
                else { pend = true; first_entry = cut; }
            }
            if (wi && !wj) { lastexit = cut_at(L, i, pi, pj, true, iso); have_exit = true; }
            pi = pj;
            wi = wj;
        }
    }
    if (pend) tri(first_entry, lastexit);
}

// The swept integral over the step of this lane's face (Eqs. dV, alphaf): the face fanned about
// its vertex mean, each triangle's submerged fraction integrated in time exactly.
template <int kFP>
__device__ double face_sweep(const Pt *P, const FaceLoop<kFP> &L, D3 xS, D3 nS, double un, double dt) {
    D3 ap{0, 0, 0};
#pragma unroll
    for (int i = 0; i < kFP; ++i)
        if (i < L.n) ap = ap + xyz(fetch(P, L, i));
    ap = (1.0 / L.n) * ap;
    const double dap = dot(ap - xS, nS);
    double accI = 0.0, Af = 0.0;
    const D3 x0 = xyz(fetch(P, L, 0));
    D3 xi = x0;
#pragma unroll
    for (int i = 0; i < kFP; ++i) {
        if (i < L.n) {
            D3 xj = x0;
            if (i + 1 < kFP && i + 1 < L.n) xj = xyz(fetch(P, L, i + 1));
            const double Ai = 0.5 * norm3(cross(xi - ap, xj - ap));
            accI += Ai * tri_sweep(dap, dot(xi - xS, nS), dot(xj - xS, nS), un, dt);
            Af += Ai;
            xi = xj;
        }
    }
    return accI / Af;
}

// kInterp: U_S by cell-point interpolation (us_mode 1): the points' velocities (the vertex values'
// inverse-distance weights) sit in LDS beside the points, and each lane tests the tetrahedra that
// fan its face about the face's mean point with the cell centroid.
template <int kFP, bool kInterp>
__global__ void __launch_bounds__(kGrp * kGrpPerBlock) k_surface_big(BigArgs A) {
    __shared__ Pt spt[kGrpPerBlock][kBigPts];
    __shared__ double ssort[kGrpPerBlock][kBigPts];
    __shared__ D3 svel[kInterp ? kGrpPerBlock : 1][kInterp ? kBigPts : 1];
    const DevMesh &m = A.m;
    const int g = threadIdx.x / kGrp, lf = threadIdx.x % kGrp;
    Pt *P = spt[g];
    double *S = ssort[g];
    const int n = min(A.counters[kCntSurf], A.cap);
    int rounds_max = 0, flat = 0, nonconv = 0;
    for (int idx = blockIdx.x * kGrpPerBlock + g; idx < n; idx += gridDim.x * kGrpPerBlock) {
        const int c = A.list[idx];
        const int bi = m.cbig[c];
        if (bi < 0) continue;  // the same cell on all sixteen lanes
        if (A.only_class >= 0 && ((m.cflags[c] >> 11) & 1) != A.only_class) continue;  // the other launch's
        const double aP = A.alpha[c];
        const double V6 = 6.0 * m.vol[c];
        const double dtc = cell_dt(m, A.dt_dom, A.dt, c);  // an ensemble member's own time step
        // points lf and lf + 16: coordinates, their mean over the group, vertex values
        const int v0 = m.bv_ptr[bi], nv = m.bv_ptr[bi + 1] - v0;
        D3 xp[2], up[2];
        double ap[2];
        D3 xs{0, 0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lf + kGrp * h;
            xp[h] = up[h] = D3{0, 0, 0};
            ap[h] = 0.0;
            if (i < nv) {
                const double *q = m.bv_xyz + 3 * (size_t)(v0 + i);
                xp[h] = D3{q[0], q[1], q[2]};
                const int k = m.bv_cls[v0 + i];
                double av = 0.0;
#pragma unroll 4
                for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e) av += m.st_w[e] * A.alpha[m.st_cell[e]];
                ap[h] = av;
                xs = xs + xp[h];
                if constexpr (kInterp) {
                    const size_t nc = m.n_cells;
                    D3 u{0, 0, 0};
                    for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e) {
                        const int32_t sc = m.st_cell[e];
                        D3 us{A.U[sc], A.U[nc + sc], A.U[2 * nc + sc]};
                        if (A.U1) us = 0.5 * (us + D3{A.U1[sc], A.U1[nc + sc], A.U1[2 * nc + sc]});
                        u = u + m.st_w[e] * us;
                    }
                    up[h] = u;
                }
            }
        }
        const D3 xm = (1.0 / nv) * g16_3(xs);
        grp_sync();  // the previous cell's reads of P and S are done
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lf + kGrp * h;
            if (i < nv) {
                const D3 x = xp[h] - xm;
                P[i] = Pt{x.x, x.y, x.z, ap[h]};
                if constexpr (kInterp) svel[g][i] = up[h];
            }
        }
        grp_sync();
        // sorted vertex values: each point's rank (ties by index)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lf + kGrp * h;
            if (i < nv) {
                int rank = 0;
                for (int j = 0; j < nv; ++j) {
                    const double aj = P[j].a;
                    rank += (aj < ap[h] || (aj == ap[h] && j < i)) ? 1 : 0;
                }
                S[rank] = ap[h];
            }
        }
        // this lane's face
        const int f0 = m.bf_ptr[bi], nf = m.bf_ptr[bi + 1] - f0;
        FaceLoop<kFP> L{};
        if (lf < nf) {
            const int b = m.bl_ptr[f0 + lf];
            L.n = m.bl_ptr[f0 + lf + 1] - b;
            L.planar = m.bf_planar[f0 + lf];
#pragma unroll
            for (int i = 0; i < kFP; ++i)
                if (i < L.n) L.w[i >> 2] |= (uint32_t)m.bl_vtx[b + i] << (8 * (i & 3));
            if constexpr (kFP <= 4) {
#pragma unroll
                for (int i = 0; i < kFP; ++i)
                    if (i < L.n) L.q[i] = P[loop_at(L, i)];
#pragma unroll
                for (int i = 0; i < kFP; ++i) {
                    const double ai = L.q[i].a, aj = (i + 1 < L.n ? L.q[(i + 1) % kFP] : L.q[0]).a;
                    L.r[i] = (i < L.n && ai != aj) ? 1.0 / (fmin(ai, aj) - fmax(ai, aj)) : 0.0;
                }
            }
        }
        grp_sync();
        // every face planar: the bracket's Newton solve
        const uint64_t pb = __ballot(L.n == 0 || L.planar != 0);
        const bool planar_cell = ((pb >> (__lane_id() & ~(kGrp - 1))) & 0xFFFFull) == 0xFFFFull;
        bool recon = S[nv - 1] - S[0] > A.flat_tol;
        double iso = 0.0;
        int rounds = 0;
        D3 nS{0, 0, 0}, xS{0, 0, 0};
        double un = 0.0;
        if (recon) {
            D3 o, cseg;
            auto F = [&](double x, bool tie_wet) { return grp_vsub6(P, L, x, tie_wet, o, cseg) / V6 - aP; };
            int il = 0, ih = nv - 1;
            double fl = 1.0 - aP;
            bool exact = false;
            while (ih - il > 1) {
                const int im = (il + ih) >> 1;
                const double fm = F(S[im], false);
                ++rounds;
                if (fm > 0.0) { il = im; fl = fm; }
                else if (fm < 0.0) { ih = im; }
                else { iso = S[im]; exact = true; break; }
            }
            if (!exact) {
                double x0 = S[il], x1 = S[ih], f0v = fl;
                double f1 = F(x1, true);  // limit from below at x1
                ++rounds;
                if (f1 > 0.0) {
                    iso = x1;  // the sub-volume jumps across alpha_P at this vertex value
                } else if (planar_cell) {
                    // Newton on the bracket's functional form (safeguarded by the bracket, a
                    // power-law step when Newton leaves it, stopped at round-off or when the
                    // change of slope shows the next step below it)
                    const double xr = x0, uhi = x1 - x0, target = aP * V6;
                    auto G = [&](double u, double &dG) {
                        const IntervalPart q = face_interval(P, L, xr, u);
                        const D3 oacc = g16_3(q.oacc), doacc = g16_3(q.doacc), Bs = g16_3(q.B), dBs = g16_3(q.dB);
                        const double oL = g16(q.oL), doL = g16(q.doL), v = g16(q.v), dv = g16(q.dv);
                        D3 oo{0, 0, 0}, od{0, 0, 0};
                        if (oL > 0.0) {
                            const double il = 1.0 / oL;
                            oo = il * oacc;
                            od = il * (doacc - doL * oo);
                        }
                        dG = dv + dot(od, Bs) + dot(oo, dBs);
                        return v + dot(oo, Bs) - target;
                    };
                    double ua = 0.0, ub = uhi, ga = f0v * V6, gb = f1 * V6;
                    double u = ua + (ub - ua) * (ga / (ga - gb));  // secant start
                    double up = uhi, dGp = 0.0;
                    bool conv = false, first = true;
                    for (; rounds < A.max_rounds; ++rounds) {
                        double dG;
                        const double g = G(u, dG);
                        if (fabs(g) <= A.root_tol * V6) { conv = true; ++rounds; break; }  // g == 0 at 0
                        if (g > 0.0) { ua = u; ga = g; } else { ub = u; gb = g; }
                        double nu = dG < 0.0 ? u - g / dG : ua;
                        const bool newton = nu > ua && nu < ub;
                        if (!newton) {
                            const bool left = ga <= -gb;
                            const double wd = (ub - ua) * cbrt((left ? ga : -gb) / (ga - gb));
                            nu = left ? ua + wd : ub - wd;
                            if (!(nu > ua && nu < ub)) nu = 0.5 * (ua + ub);
                        }
                        const double tolu = 2.0 * __DBL_EPSILON__ * fmax(fabs(xr + nu), 1e-300);
                        const double st = nu - u;
                        bool done = fabs(st) <= tolu;
                        if (newton && !done && !first && fabs(st) <= 1e-3 * uhi)
                            done = fabs(dG - dGp) * st * st <= 0.25 * tolu * fabs(dG) * fabs(u - up);
                        up = u;
                        dGp = dG;
                        u = nu;
                        first = false;
                        if (done || !(ub - ua > 2.0 * __DBL_EPSILON__ * fmax(fabs(xr + ua), fabs(xr + ub)))) {
                            conv = true;
                            ++rounds;
                            break;
                        }
                    }
                    if (!conv) ++nonconv;
                    iso = xr + u;
                } else {
                    int side = 0;
                    bool conv = false;
                    for (; rounds < A.max_rounds; ++rounds) {
                        const double wdt = x1 - x0;
                        if (!(wdt > 4.0 * __DBL_EPSILON__ * fmax(fabs(x0), fabs(x1)))) { conv = true; break; }
                        double x = x1 - f1 * (x1 - x0) / (f1 - f0v);
                        if (!(x > x0 && x < x1) || (rounds & 7) == 7) x = x0 + 0.5 * wdt;
                        const double fx = F(x, false);
                        if (fabs(fx) <= fmax(4.0 * __DBL_EPSILON__, A.root_tol)) {
                            x0 = x1 = x;
                            f0v = f1 = fx;
                            conv = true;
                            ++rounds;
                            break;
                        }
                        if (fx > 0.0) {
                            x0 = x; f0v = fx;
                            if (side == 1) f1 *= 0.5;
                            side = 1;
                        } else {
                            x1 = x; f1 = fx;
                            if (side == -1) f0v *= 0.5;
                            side = -1;
                        }
                    }
                    if (!conv) ++nonconv;
                    iso = fabs(f0v) <= fabs(f1) ? x0 : x1;
                }
            }
            // the isoface at the isovalue: normal from its area vector, centre from its fan
            grp_vsub6(P, L, iso, false, o, cseg);
            const double nrm = norm3(cseg);
            if (nrm > 0.0) {
                nS = (1.0 / nrm) * cseg;
                D3 acc;
                double ws;
                face_centre(P, L, iso, o, nS, acc, ws);
                acc = g16_3(acc);
                ws = g16(ws);
                xS = (1.0 / (3.0 * ws)) * acc;
                const size_t nc = m.n_cells;
                D3 Up{A.U[c], A.U[nc + c], A.U[2 * nc + c]};
                if (A.U1) Up = 0.5 * (Up + D3{A.U1[c], A.U1[nc + c], A.U1[2 * nc + c]});
                D3 Us = Up;
                if constexpr (kInterp) {
                    // each lane keeps the tetrahedron of its face whose smallest barycentric
                    // coordinate of x_S (Cramer's rule) is largest; the group takes the best
                    // (lowest lane on a tie)
                    const D3 cc = D3{m.ccen[3 * (size_t)c], m.ccen[3 * (size_t)c + 1], m.ccen[3 * (size_t)c + 2]} - xm;
                    const D3 *Uv = svel[g];
                    double best = -INFINITY;
                    D3 val = Up;
                    if (lf < nf) {
                        // loop positions as compile-time indices where the face's points are held
                        // in registers (faces of at most four points)
                        constexpr int kMax = kFP <= 4 ? 4 : kFP;
                        D3 fc{0, 0, 0}, uf{0, 0, 0};
#pragma unroll
                        for (int i = 0; i < kMax; ++i) {
                            if (i < L.n) {
                                const Pt q = fetch(P, L, i);
                                fc = fc + D3{q.x, q.y, q.z};
                                uf = uf + Uv[loop_at(L, i)];
                            }
                        }
                        fc = (1.0 / L.n) * fc;
                        uf = (1.0 / L.n) * uf;
                        const D3 e1 = fc - cc, r = xS - cc;
                        const Pt q0 = fetch(P, L, 0);
#pragma unroll
                        for (int i = 0; i < kMax; ++i) {
                            if (i >= L.n) continue;
                            const Pt qi = fetch(P, L, i);
                            const Pt qj = i + 1 < L.n ? fetch(P, L, i + 1 < kMax ? i + 1 : 0) : q0;
                            const int j = i + 1 < L.n ? i + 1 : 0;
                            const D3 e2 = D3{qi.x, qi.y, qi.z} - cc, e3 = D3{qj.x, qj.y, qj.z} - cc;
                            const D3 k23 = cross(e2, e3);
                            const double det = dot(e1, k23);
                            if (det == 0.0) continue;
                            const double l1 = dot(r, k23) / det, l2 = dot(e1, cross(r, e3)) / det,
                                         l3 = dot(e1, cross(e2, r)) / det;
                            const double l0 = 1.0 - l1 - l2 - l3;
                            const double mn = fmin(fmin(l0, l1), fmin(l2, l3));
                            if (mn > best) {
                                best = mn;
                                val = l0 * Up + l1 * uf + l2 * Uv[loop_at(L, i)] + l3 * Uv[loop_at(L, j)];
                            }
                        }
                    }
                    double gb = best;
#pragma unroll
                    for (int off = 1; off < kGrp; off <<= 1) gb = fmax(gb, __shfl_xor(gb, off, kGrp));
                    const uint64_t bal = __ballot(best == gb);
                    const uint32_t gm = (uint32_t)(bal >> (__lane_id() & ~(kGrp - 1))) & 0xFFFFu;
                    const int win = __ffs(gm) - 1;
                    Us = D3{__shfl(val.x, win, kGrp), __shfl(val.y, win, kGrp), __shfl(val.z, win, kGrp)};
                }
                un = dot(Us, nS);
            } else {
                recon = false;
            }
        }
        if (lf == 0) {
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
        }
        // this lane's face, if it carries outflow
        if (lf < nf) {
            const int32_t v = m.bf_face[f0 + lf];
            if (v != kEmpty) {
                const int32_t fid = v >= 0 ? v : ~v;
                const double ph = A.phi1 ? 0.5 * (A.phi[fid] + A.phi1[fid]) : A.phi[fid];
                const double out = v >= 0 ? ph : -ph;
                if (out > 0.0) A.dvs[fid] = recon ? ph * face_sweep(P, L, xS, nS, un, dtc) : aP * ph * dtc;
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
            // every lane of a group counts its cell's search: one count per group
            if (nonconv) atomicAdd(&A.counters[kCntNonconv], nonconv / kGrp);
        }
    }
}

}  // namespace

hipError_t launch_surface_big(const BigArgs &a, hipStream_t s) {
    const int blocks = std::max(1, std::min(1024, (a.cap + kGrpPerBlock - 1) / kGrpPerBlock));
    const dim3 g(blocks), b(kGrp * kGrpPerBlock);
    // a single mesh: the instantiation its largest face needs; an ensemble whose members need
    // both: one launch of each, each taking its own members' polyhedra (as each member alone)
    auto launch = [&](bool wide, int only) {
        BigArgs x = a;
        x.only_class = only;
        if (!wide) {
            if (x.us_mode == 1) hipLaunchKernelGGL((k_surface_big<4, true>), g, b, 0, s, x);
            else hipLaunchKernelGGL((k_surface_big<4, false>), g, b, 0, s, x);
        } else {
            if (x.us_mode == 1) hipLaunchKernelGGL((k_surface_big<kBigFacePts, true>), g, b, 0, s, x);
            else hipLaunchKernelGGL((k_surface_big<kBigFacePts, false>), g, b, 0, s, x);
        }
    };
    if (a.m.big_class == 2) {
        launch(false, 0);
        launch(true, 1);
    } else {
        launch(a.m.big_face_pts > 4, -1);
    }
    return hipGetLastError();
}

}  // namespace isoadv
