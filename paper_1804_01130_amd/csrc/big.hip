// Interface cells of general polyhedra (Section 3: arbitrary polyhedral control volumes; Section
// 3.2: the isoface construction on them): cells beyond what the eight-lane kernel takes (more
// than six faces, more than eight points, or faces of more than four points), up to kBigPts
// points, kBigFaces faces and kBigFacePts points per face.
//
// One thread per such cell, grid-stride over the interface-cell list (the other cells are left to
// the eight-lane kernel, which skips these).  The thread follows the same construction as the
// eight-lane kernel's generic path, with loops over the cell's faces and each face's points:
//   vertex values through the inverse-distance stencils; the isovalue bracketed between two
//   consecutive sorted vertex values (the limit from above at each) and found by Illinois with a
//   bisection guard to round-off, or taken at a vertex value where the sub-volume jumps; the
//   sub-volume by the divergence theorem, each face's wet loop fanned about a face point (planar
//   faces) or its perimeter centroid, the isoface fanned about the perimeter centroid of its
//   edges; the isoface's normal, centre and U_P . n_S; and for each outflow face the swept
//   integral over the triangles that fan the face about its vertex mean.
// These cells are expected to be few (hexahedra-dominant meshes), so the work is laid out for
// clarity: the cell's points and values wait in the thread's private memory, its face loops are
// read where they lie.
#include "device_common.h"
#include "internal.h"

namespace isoadv {

namespace {

struct BigPart {
    double v6;
    D3 cseg, oacc;
    double oL;
};

struct BigCell {
    int nv, nf;
    D3 x[kBigPts];         // points relative to their mean
    double a[kBigPts];     // vertex values
    const int32_t *fptr;   // [nf+1] loop positions of each face (offsets into loop)
    const int32_t *loop;   // local point at each loop position
    const int32_t *planar; // [nf]
};

// Cut point on the edge from point p to point q of a face: from the wet end, so that the two faces
// sharing the edge compute the same point.
__device__ __forceinline__ D3 big_cut(const BigCell &B, int p, int q, bool wet_p, double iso) {
    const int w = wet_p ? p : q, d = wet_p ? q : p;
    const double lam = (iso - B.a[w]) / (B.a[d] - B.a[w]);
    return B.x[w] + lam * (B.x[d] - B.x[w]);
}

// Face k's share of six times the wet sub-volume and of the isoface sums (as the eight-lane
// kernel's face share, for any number of points).
__device__ BigPart big_face_part(const BigCell &B, int k, double iso, bool tie_wet) {
    BigPart r{0.0, {0, 0, 0}, {0, 0, 0}, 0.0};
    const int b = B.fptr[k], n = B.fptr[k + 1] - b;
    auto wet = [&](int i) {
        const double av = B.a[B.loop[b + i]];
        return tie_wet ? av >= iso : av > iso;
    };
    // the last exit before the start of the loop
    D3 lastexit{0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const int j = i + 1 < n ? i + 1 : 0;
        if (wet(i) && !wet(j)) lastexit = big_cut(B, B.loop[b + i], B.loop[b + j], true, iso);
    }
    D3 C{0, 0, 0}, pacc{0, 0, 0}, psum{0, 0, 0};
    double pl = 0.0;
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
        const int j = i + 1 < n ? i + 1 : 0;
        const int p = B.loop[b + i], q = B.loop[b + j];
        const bool wi = wet(i), wj = wet(j);
        const D3 cut = big_cut(B, p, q, wi, iso);
        if (!wi && wj) {  // an entry: the isoface edge from here back to the preceding exit
            const D3 s0 = cut, s1 = lastexit;
            const double l = norm3(s1 - s0);
            r.cseg = r.cseg + cross(s0, s1);
            r.oacc = r.oacc + (0.5 * l) * (s0 + s1);
            r.oL += l;
        }
        if (wi && !wj) lastexit = cut;
        if (wi || wj) {
            const D3 u = wi ? B.x[p] : cut, v = wj ? B.x[q] : cut;
            C = C + cross(u, v);
            const double l = norm3(v - u);
            pacc = pacc + (0.5 * l) * (u + v);
            pl += l;
        }
        if (wi) psum = psum + B.x[p];
        if (wi != wj) psum = psum + cut;
        cnt += (wi ? 1 : 0) + (wi != wj ? 1 : 0);
    }
    C = C - r.cseg;  // the isoface edges close the wet loop, walked exit to entry
    if (cnt >= 3) {
        D3 ap = B.x[B.loop[b]];
        if (!B.planar[k]) {
            const D3 tot = pacc + r.oacc;
            const double tl = pl + r.oL;
            ap = tl > 0.0 ? (1.0 / tl) * tot : (1.0 / cnt) * psum;
        }
        r.v6 = dot(ap, C);
    }
    return r;
}

__device__ double big_vsub6(const BigCell &B, double iso, bool tie_wet, D3 *o_out, D3 *cseg_out) {
    double v6 = 0.0, oL = 0.0;
    D3 cseg{0, 0, 0}, oacc{0, 0, 0};
    for (int k = 0; k < B.nf; ++k) {
        const BigPart p = big_face_part(B, k, iso, tie_wet);
        v6 += p.v6;
        cseg = cseg + p.cseg;
        oacc = oacc + p.oacc;
        oL += p.oL;
    }
    const D3 o = oL > 0.0 ? (1.0 / oL) * oacc : D3{0, 0, 0};
    if (o_out) *o_out = o;
    if (cseg_out) *cseg_out = cseg;
    return v6 + dot(o, cseg);
}

__global__ void __launch_bounds__(64) k_surface_big(BigArgs A) {
    const DevMesh &m = A.m;
    const int n = min(A.counters[kCntSurf], A.cap);
    int rounds_max = 0, flat = 0, nonconv = 0;
    BigCell B;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
        const int c = A.list[idx];
        const int bi = m.cbig[c];
        if (bi < 0) continue;
        const double aP = A.alpha[c];
        const double V6 = 6.0 * m.vol[c];
        const double dtc = A.dt;
        // the cell's points, relative to their mean, and their values through the stencils
        const int v0 = m.bv_ptr[bi];
        B.nv = m.bv_ptr[bi + 1] - v0;
        D3 xm{0, 0, 0};
        for (int i = 0; i < B.nv; ++i) {
            B.x[i] = D3{m.bv_xyz[3 * (size_t)(v0 + i)], m.bv_xyz[3 * (size_t)(v0 + i) + 1],
                        m.bv_xyz[3 * (size_t)(v0 + i) + 2]};
            xm = xm + B.x[i];
        }
        xm = (1.0 / B.nv) * xm;
        for (int i = 0; i < B.nv; ++i) {
            B.x[i] = B.x[i] - xm;
            const int k = m.bv_cls[v0 + i];
            double av = 0.0;
            for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e) av += m.st_w[e] * A.alpha[m.st_cell[e]];
            B.a[i] = av;
        }
        const int f0 = m.bf_ptr[bi];
        B.nf = m.bf_ptr[bi + 1] - f0;
        B.fptr = m.bl_ptr + f0;  // loop positions of face k: [fptr[k], fptr[k+1]) of bl_vtx
        B.loop = m.bl_vtx;
        B.planar = m.bf_planar + f0;
        // sorted vertex values (insertion sort)
        double s[kBigPts];
        for (int i = 0; i < B.nv; ++i) {
            double v = B.a[i];
            int j = i;
            while (j > 0 && s[j - 1] > v) { s[j] = s[j - 1]; --j; }
            s[j] = v;
        }
        bool recon = s[B.nv - 1] - s[0] > A.flat_tol;
        double iso = 0.0;
        int rounds = 0;
        D3 nS{0, 0, 0}, xS{0, 0, 0};
        double un = 0.0;
        if (recon) {
            auto F = [&](double x, bool tie_wet) { return big_vsub6(B, x, tie_wet, nullptr, nullptr) / V6 - aP; };
            int il = 0, ih = B.nv - 1;
            double fl = 1.0 - aP;
            bool exact = false;
            while (ih - il > 1) {
                const int im = (il + ih) >> 1;
                const double fm = F(s[im], false);
                ++rounds;
                if (fm > 0.0) { il = im; fl = fm; }
                else if (fm < 0.0) { ih = im; }
                else { iso = s[im]; exact = true; break; }
            }
            if (!exact) {
                double x0 = s[il], x1 = s[ih], f0v = fl;
                double f1 = F(x1, true);  // limit from below at x1
                ++rounds;
                if (f1 > 0.0) {
                    iso = x1;  // the sub-volume jumps across alpha_P at this vertex value
                } else {
                    int side = 0;
                    bool conv = false;
                    for (; rounds < A.max_rounds; ++rounds) {
                        const double wdt = x1 - x0;
                        if (!(wdt > 4.0 * __DBL_EPSILON__ * fmax(fabs(x0), fabs(x1)))) { conv = true; break; }
                        double x = x1 - f1 * (x1 - x0) / (f1 - f0v);
                        if (!(x > x0 && x < x1) || (rounds & 7) == 7) x = x0 + 0.5 * wdt;
                        const double fx = F(x, false);
                        if (fx == 0.0 || fabs(fx) <= 4.0 * __DBL_EPSILON__) {
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
            D3 o, cseg;
            big_vsub6(B, iso, false, &o, &cseg);
            const double nrm = norm3(cseg);
            if (nrm > 0.0) {
                nS = (1.0 / nrm) * cseg;
                D3 acc{0, 0, 0};
                double ws = 0.0;
                for (int k = 0; k < B.nf; ++k) {
                    const int b = B.fptr[k], nn = B.fptr[k + 1] - b;
                    auto wet = [&](int i) { return B.a[B.loop[b + i]] > iso; };
                    D3 lastexit{0, 0, 0};
                    for (int i = 0; i < nn; ++i) {
                        const int j = i + 1 < nn ? i + 1 : 0;
                        if (wet(i) && !wet(j)) lastexit = big_cut(B, B.loop[b + i], B.loop[b + j], true, iso);
                    }
                    for (int i = 0; i < nn; ++i) {
                        const int j = i + 1 < nn ? i + 1 : 0;
                        const bool wi = wet(i), wj = wet(j);
                        const D3 cut = big_cut(B, B.loop[b + i], B.loop[b + j], wi, iso);
                        if (!wi && wj) {
                            const double wt = dot(cross(cut - o, lastexit - o), nS);
                            acc = acc + wt * (o + cut + lastexit);
                            ws += wt;
                        }
                        if (wi && !wj) lastexit = cut;
                    }
                }
                xS = (1.0 / (3.0 * ws)) * acc;
                const size_t nc = m.n_cells;
                D3 Up{A.U[c], A.U[nc + c], A.U[2 * nc + c]};
                if (A.U1) Up = 0.5 * (Up + D3{A.U1[c], A.U1[nc + c], A.U1[2 * nc + c]});
                un = dot(Up, nS);
            } else {
                recon = false;
            }
        }
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
        // outflow faces: the swept integral over the triangles fanning each face about its
        // vertex mean (a planar face's fan covers it whatever the apex)
        for (int k = 0; k < B.nf; ++k) {
            const int32_t v = m.bf_face[f0 + k];
            if (v == kEmpty) continue;
            const int32_t fid = v >= 0 ? v : ~v;
            const double ph = A.phi1 ? 0.5 * (A.phi[fid] + A.phi1[fid]) : A.phi[fid];
            const double out = v >= 0 ? ph : -ph;
            if (!(out > 0.0)) continue;
            double dv;
            if (recon) {
                const int b = B.fptr[k], nn = B.fptr[k + 1] - b;
                D3 ap{0, 0, 0};
                for (int i = 0; i < nn; ++i) ap = ap + B.x[B.loop[b + i]];
                ap = (1.0 / nn) * ap;
                const double dap = dot(ap - xS, nS);
                double accI = 0.0, Af = 0.0;
                for (int i = 0; i < nn; ++i) {
                    const D3 p = B.x[B.loop[b + i]], q = B.x[B.loop[b + (i + 1 < nn ? i + 1 : 0)]];
                    const double Ai = 0.5 * norm3(cross(p - ap, q - ap));
                    accI += Ai * tri_sweep(dap, dot(p - xS, nS), dot(q - xS, nS), un, dtc);
                    Af += Ai;
                }
                dv = ph * (accI / Af);
            } else {
                dv = aP * ph * dtc;
            }
            A.dvs[fid] = dv;
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
            if (nonconv) atomicAdd(&A.counters[kCntNonconv], nonconv);
        }
    }
}

}  // namespace

hipError_t launch_surface_big(const BigArgs &a, hipStream_t s) {
    const int blocks = std::max(1, std::min(256, (a.cap + 63) / 64));
    hipLaunchKernelGGL(k_surface_big, dim3(blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace isoadv
