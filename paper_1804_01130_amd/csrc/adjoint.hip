// Adjoint (vector-Jacobian product) of one isoAdvector step on gfx950, FP64.
//
// Given the adjoint of alpha_new, the step's inputs and its intermediates (vertex values, cell
// kinds, isovalues, face volumes dV and the update before bounding, as the traced forward step
// writes them), these launches produce the adjoints of alpha and phi:
//   prep       per cell: the update's round-off chop, the cells the bounding sweeps start from
//              (and their first corrections); per face buffers cleared
//   sweep      one per bounding sweep, grid-wide: the sweeps replayed with a tape (same
//              arithmetic as the forward)
//   unsweep    two per sweep, in reverse: the bounding step (end of Section 3.2) transposed
//   faces      per cell, a gather over its flux faces: transposes of the flux-form update and of
//              the bulk fluxes alpha_upwind phi dt; phi's adjoint through dV = phi * (dV/phi); and
//              the interface cells' directions (their isovalue, and each vertex value a cut edge
//              touches)
//   surface    eight lanes per (interface cell, direction): rates of the sub-volume and of the
//              swept face integrals (Eqs. tv .. intaplus) by forward-mode dual numbers through
//              the isoface
//   points     per point class, and cells, per cell: the isovalue moving with the volume
//              constraint (implicit function) combines the rates, and the transpose of the
//              vertex interpolation gathers them to the stencil cells in a fixed order
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"

namespace isoadv {
namespace {

// ------------------------------------------------------------------------------- dual numbers
struct Dl {
    double v, d;  // value and derivative along one direction
};
__device__ __forceinline__ Dl operator+(Dl a, Dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dl operator-(Dl a, Dl b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dl operator-(Dl a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dl operator*(Dl a, Dl b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dl operator*(double s, Dl a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dl operator/(Dl a, Dl b) {
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dl dinv(Dl a) {
    const double q = 1.0 / a.v;
    return {q, -a.d * q * q};
}
__device__ __forceinline__ Dl dsqrt(Dl a) {
    const double r = sqrt(a.v);
    return {r, r > 0.0 ? 0.5 * a.d / r : 0.0};
}
__device__ __forceinline__ Dl dsel(bool c, Dl a, Dl b) { return {c ? a.v : b.v, c ? a.d : b.d}; }
__device__ __forceinline__ Dl dc(double x) { return {x, 0.0}; }

struct DV3 {
    Dl x, y, z;
};
__device__ __forceinline__ DV3 operator+(DV3 a, DV3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ DV3 operator-(DV3 a, DV3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ DV3 operator*(Dl s, DV3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ DV3 operator*(double s, DV3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ DV3 dv(D3 a) { return {dc(a.x), dc(a.y), dc(a.z)}; }
__device__ __forceinline__ Dl ddot(DV3 a, DV3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ DV3 dcross(DV3 a, DV3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ Dl dnorm(DV3 a) { return dsqrt(ddot(a, a)); }
__device__ __forceinline__ DV3 dsel3(bool c, DV3 a, DV3 b) { return {dsel(c, a.x, b.x), dsel(c, a.y, b.y), dsel(c, a.z, b.z)}; }
__device__ __forceinline__ Dl dgrp_sum(Dl a) { return {grp_sum(a.v), grp_sum(a.d)}; }
__device__ __forceinline__ DV3 dgrp_sum3(DV3 a) { return {dgrp_sum(a.x), dgrp_sum(a.y), dgrp_sum(a.z)}; }

// A lane's face with dual vertex values (geometry is fixed).
struct DFace {
    D3 q[4];
    Dl aq[4];
    Dl inv[4];
    int fwd;
    bool planar, active;
};

__device__ __forceinline__ DV3 dface_cut(const DFace &f, int i, Dl iso, bool wet_i) {
    const int j = (i + 1) & 3;
    const bool fwd = (f.fwd >> i) & 1;
    const D3 xw = sel3(wet_i, f.q[i], f.q[j]), xd = sel3(wet_i, f.q[j], f.q[i]);
    const Dl aw = dsel(wet_i, f.aq[i], f.aq[j]);
    const Dl lam = (wet_i == fwd) ? (iso - aw) * f.inv[i] : (aw - iso) * f.inv[i];
    return dv(xw) + lam * dv(xd - xw);
}

struct DPart {
    Dl v6;
    DV3 cseg, oacc;
    Dl oL;
    DV3 osum;
    double nseg;
};

// The face's share of six times the sub-volume and of the isoface sums (the same construction as
// the forward kernel, in dual numbers; wet iff a > iso).
__device__ __forceinline__ DPart dface_part(const DFace &f, Dl iso) {
    const DV3 Z = dv(D3{0, 0, 0});
    DPart r{dc(0.0), Z, Z, dc(0.0), Z, 0.0};
    bool w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = f.active && f.aq[i].v > iso.v;
    DV3 cut[4];
    bool cuts[4], exits[4], entries[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        cut[i] = dface_cut(f, i, iso, w[i]);
        cuts[i] = w[i] != w[j];
        exits[i] = w[i] && !w[j];
        entries[i] = !w[i] && w[j];
    }
    DV3 last = Z;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        last = dsel3(w[i], dv(f.q[i]), last);
        last = dsel3(cuts[i], cut[i], last);
        cnt += (w[i] ? 1 : 0) + (cuts[i] ? 1 : 0);
    }
    DV3 C = Z, prev = last;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        C = dsel3(w[i], C + dcross(prev, dv(f.q[i])), C);
        prev = dsel3(w[i], dv(f.q[i]), prev);
        C = dsel3(cuts[i], C + dcross(prev, cut[i]), C);
        prev = dsel3(cuts[i], cut[i], prev);
    }
    if (cnt >= 3) {
        DV3 ap = dv(f.q[0]);
        if (!f.planar) {
            DV3 pacc = Z, psum = Z, pv = last;
            Dl pl = dc(0.0);
            auto step = [&](bool on, DV3 x) {
                const Dl l = dnorm(x - pv);
                pacc = dsel3(on, pacc + (0.5 * l) * (x + pv), pacc);
                pl = dsel(on, pl + l, pl);
                psum = dsel3(on, psum + x, psum);
                pv = dsel3(on, x, pv);
            };
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                step(w[i], dv(f.q[i]));
                step(cuts[i], cut[i]);
            }
            ap = pl.v > 0.0 ? dinv(pl) * pacc : (1.0 / cnt) * psum;
        }
        r.v6 = ddot(ap, C);
    }
    DV3 lastexit = Z;
#pragma unroll
    for (int i = 0; i < 4; ++i) lastexit = dsel3(exits[i], cut[i], lastexit);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const DV3 s0 = cut[i], s1 = lastexit;
        if (entries[i]) {
            const Dl l = dnorm(s1 - s0);
            r.cseg = r.cseg + dcross(s0, s1);
            r.oacc = r.oacc + (0.5 * l) * (s0 + s1);
            r.oL = r.oL + l;
            r.osum = r.osum + s0;
            r.nseg += 1.0;
        }
        lastexit = dsel3(exits[i], cut[i], lastexit);
    }
    return r;
}

// Six times the sub-volume (all lanes of the group), and the isoface apex and area vector (x2).
__device__ __forceinline__ Dl dcell_vsub6(const DFace &f, Dl iso, DV3 *o_out, DV3 *cseg_out) {
    const DPart p = dface_part(f, iso);
    const Dl v6 = dgrp_sum(p.v6);
    const DV3 cseg = dgrp_sum3(p.cseg), oacc = dgrp_sum3(p.oacc), osum = dgrp_sum3(p.osum);
    const Dl oL = dgrp_sum(p.oL);
    const double nseg = grp_sum(p.nseg);
    const DV3 Z = dv(D3{0, 0, 0});
    const DV3 o = oL.v > 0.0 ? dinv(oL) * oacc : (nseg > 0.0 ? (1.0 / nseg) * osum : Z);
    if (o_out) *o_out = o;
    if (cseg_out) *cseg_out = cseg;
    return v6 + ddot(o, cseg);
}

__device__ __forceinline__ void dface_centre_part(const DFace &f, Dl iso, DV3 o, DV3 n, DV3 &acc, Dl &ws) {
    const DV3 Z = dv(D3{0, 0, 0});
    acc = Z;
    ws = dc(0.0);
    bool w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = f.active && f.aq[i].v > iso.v;
    DV3 cut[4];
    bool exits[4], entries[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) & 3;
        cut[i] = dface_cut(f, i, iso, w[i]);
        exits[i] = w[i] && !w[j];
        entries[i] = !w[i] && w[j];
    }
    DV3 lastexit = Z;
#pragma unroll
    for (int i = 0; i < 4; ++i) lastexit = dsel3(exits[i], cut[i], lastexit);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const DV3 s0 = cut[i], s1 = lastexit;
        if (entries[i]) {
            const Dl wt = ddot(dcross(s0 - o, s1 - o), n);
            acc = acc + wt * (o + s0 + s1);
            ws = ws + wt;
        }
        lastexit = dsel3(exits[i], cut[i], lastexit);
    }
}

// Swept integral of a triangle (the forward kernel's construction in dual numbers): the wet
// fraction at time s is the area distribution of the distances at un*s; breakpoints clamped to
// the window; each piece integrated exactly (Simpson) on the branch of its midpoint.
__device__ __forceinline__ Dl dtri_piece(int br, Dl z, Dl e1, Dl e2, Dl e3, Dl r31, Dl r21, Dl r32) {
    if (br == 0) return dc(0.0);
    if (br == 3) return dc(1.0);
    if (br == 1) {
        const Dl u = z - e1;
        return (u * r31) * (u * r21);
    }
    const Dl u = e3 - z;
    return dc(1.0) - (u * r31) * (u * r32);
}

__device__ __forceinline__ Dl dtri_sweep(Dl d0, Dl d1, Dl d2, Dl un, double dt) {
    // sorted by compare-and-swap: a permutation, so at a tie each distance keeps its own rate
    // (a min and a max that both return the same member would count one vertex twice)
    Dl e1 = d0, e2 = d1, e3 = d2;
    auto order = [](Dl &x, Dl &y) {
        if (y.v < x.v) {
            const Dl t = x;
            x = y;
            y = t;
        }
    };
    order(e1, e2);
    order(e2, e3);
    order(e1, e2);
    const Dl r31 = e3.v > e1.v ? dinv(e3 - e1) : dc(0.0);
    const Dl r21 = e2.v > e1.v ? dinv(e2 - e1) : dc(0.0);
    const Dl r32 = e3.v > e2.v ? dinv(e3 - e2) : dc(0.0);
    auto branch = [&](double z) { return z < e1.v ? 0 : (z < e2.v ? 1 : (z < e3.v ? 2 : 3)); };
    if (un.v == 0.0) {
        const int br = branch(0.0);
        const Dl m = un * dc(0.5 * dt), b = un * dc(dt);
        return (dt / 6.0) * (dtri_piece(br, dc(0.0), e1, e2, e3, r31, r21, r32) +
                             4.0 * dtri_piece(br, m, e1, e2, e3, r31, r21, r32) +
                             dtri_piece(br, b, e1, e2, e3, r31, r21, r32));
    }
    const Dl inv = dinv(un);
    Dl s1 = e1 * inv, s2 = e2 * inv, s3 = e3 * inv;
    if (un.v < 0.0) {
        const Dl t = s1;
        s1 = s3;
        s3 = t;
    }
    const Dl bk[3] = {s1, s2, s3};
    Dl acc = dc(0.0), a0 = dc(0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Dl a1 = dc(dt);
        if (k < 3) a1 = bk[k].v <= 0.0 ? dc(0.0) : (bk[k].v >= dt ? dc(dt) : bk[k]);
        if (a1.v > a0.v) {
            const Dl m = 0.5 * (a0 + a1);
            const int br = branch(un.v * m.v);
            const Dl fa = dtri_piece(br, un * a0, e1, e2, e3, r31, r21, r32);
            const Dl fm = dtri_piece(br, un * m, e1, e2, e3, r31, r21, r32);
            const Dl fb = dtri_piece(br, un * a1, e1, e2, e3, r31, r21, r32);
            acc = acc + (1.0 / 6.0) * ((a1 - a0) * (fa + 4.0 * fm + fb));
            a0 = a1;
        }
    }
    return acc;
}

// ------------------------------------------------------------------------------------ kernels
// A chop or clamp that moves a value by at most this much only removes round-off (which side of a
// bound such a value lands on is decided by rounding order): its derivative passes through.  A
// larger one makes the value a constant.
constexpr double kRound = 1e-14;
constexpr uint64_t kCorrBit = 1ull << 3, kTouchedBit = 1ull << 19;  // bounding tape flags, slot k: << k

// General polyhedra: sixteen lanes per (polyhedron, direction); directions 0 .. 31 are point
// values, kBigIsoDir the isovalue; per polyhedron the rates G at [0, kBigIsoDir], C at kBigC + the
// same, then the jump and 6V (see k_adj_surface_big).
constexpr int kBGrp = 16, kBGrpPerBlock = 16, kBPts = 32;
constexpr int kBigIsoDir = 32, kBigC = 33, kBigJump = 66, kBigV6 = 67;
static_assert(kAdjGBig == 68, "per-polyhedron rates: 33 + 33 + 2");

// The update's round-off chop (a move of at most the bounding tolerance) passes the derivative
// unless it moves the value by more than kRound: then the update is a constant there.
__device__ __forceinline__ bool raw_chopped(double x, int clip, double tol) {
    return clip && ((x < -kRound && x >= -tol) || (x > 1.0 + kRound && x <= 1.0 + tol));
}

struct AdjArgs {
    DevMesh m;
    const double *alpha, *phi, *U;
    double dt;
    const double *dt_dom;
    double eps, tol;
    int clip, n_iter;
    // forward intermediates of this step
    const double *vert_alpha;  // [8 nc] (interface cells)
    const int32_t *kind;       // [nc]
    const double *iso;         // [nc] (reconstructed cells)
    const double *dV0;         // [nf] dV before bounding, per flux face
    const double *raw;         // [nc] update before chopping
    // adjoint in / out
    const double *abar_new;  // [nc]
    double *abar;            // [nc]
    double *phibar;          // [nf]
    AdjWork w;
};

// Bounding replayed with a tape, then reversed, grid-wide: one kernel per forward sweep (phase B of
// sweep s fused with phase A of sweep s+1, as in the step's own sweeps; phase A of sweep 0 runs in
// k_adj_prep) and two per reversed sweep.  Tape per sweep s and listed cell (row s*nc + i, i its
// place in the sweep's list): a, need, sumcap, r, then cap and dV-now per slot; flags (64 bits, for
// up to 16 slots): bit 0 over, bit 1 r capped at 1, bit 2 sumcap > 0, bit 3+k slot k corrected, bit
// 19+k slot k read the running dV (corrected in an earlier sweep).  List order never affects a result: each listed cell writes
// only its own outflow faces and its own tape row, each touched cell only itself.
//
// Buffers that start every call at zero and are left so: the face marks (`touched`), two banks of
// cell marks (sweep s uses bank s&1: phase B of sweep s clears what phase A of sweep s+1 sets in the
// other bank), and three rotating correction buffers (sweep s writes s%3, the kernel of sweep s+1
// reads it and clears s-1's).

// Phase A of sweep s for listed cell P, row `row` of the sweep's list, with bounding state a: the
// correction of each outflow face and the tape row; the cells it touches come back through tsel.
template <int W>
__device__ __forceinline__ void adj_correct(const AdjArgs &A, int s, int32_t P, int row, double a, int32_t *mark,
                                            int32_t tsel[W + 1]) {
    constexpr int R = 4 + 2 * W;
    const int n = A.m.n_cells, nf = A.m.n_faces;
    const DevMesh &m = A.m;
    const AdjWork &w = A.w;
    const bool over = a > 1.0 + A.tol;
    const double dtc = cell_dt(m, A.dt_dom, A.dt, P);
    int32_t v[W], fid[W];
    double ph[W], cap[W], dvnow[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        v[k] = m.slot_pair[(size_t)P * W + k].x;
        fid[k] = v[k] >= 0 ? v[k] : ~v[k];
        ph[k] = v[k] != kEmpty ? A.phi[fid[k]] : 0.0;
    }
    uint64_t flags = over ? 1 : 0;
    double sumcap = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        cap[k] = 0.0;
        dvnow[k] = 0.0;
        if (v[k] == kEmpty) continue;
        const double outphi = v[k] >= 0 ? ph[k] : -ph[k];
        if (!(outphi > 0.0)) continue;
        const bool tch = w.touched[fid[k]] != 0;
        if (tch) flags |= kTouchedBit << k;
        dvnow[k] = tch ? w.dvcur[fid[k]] : A.dV0[fid[k]];
        const double outv = v[k] >= 0 ? dvnow[k] : -dvnow[k];
        cap[k] = over ? outphi * dtc - outv : outv;
        if (cap[k] > 0.0) sumcap += cap[k];
    }
    const double need = over ? (a - 1.0) * m.vol[P] : -a * m.vol[P];
    double r = 0.0;
    if (sumcap > 0.0) {
        flags |= 4;
        const double q = need / sumcap;
        if (q > 1.0) flags |= 2;
        r = fmin(q, 1.0);
    }
    if (atomicExch(&mark[P], 1) == 0) tsel[W] = P;
    double *delta = w.delta + (size_t)(s % 3) * nf;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        if (!(sumcap > 0.0) || !(cap[k] > 0.0)) continue;
        flags |= kCorrBit << k;
        const double d = cap[k] * r;
        const double dd = over ? (v[k] >= 0 ? d : -d) : (v[k] >= 0 ? -d : d);
        delta[fid[k]] = dd;
        w.dvcur[fid[k]] = dvnow[k] + dd;
        w.touched[fid[k]] = 1;
        const int32_t o = m.slot_pair[(size_t)P * W + k].y;
        if (o >= 0 && atomicExch(&mark[o], 1) == 0) tsel[k] = o;
    }
    double *rec = w.tape + ((size_t)s * n + row) * R;
    rec[0] = a;
    rec[1] = need;
    rec[2] = sumcap;
    rec[3] = r;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        rec[4 + k] = cap[k];
        rec[4 + W + k] = dvnow[k];
    }
    w.tflag[(size_t)s * n + row] = flags;
}

// Append `count` entries per thread to a device-wide list with one atomic per work-group (whole
// waves, at most 1024 threads, every one of which calls it).  Returns the index of this thread's first entry.
__device__ __forceinline__ int block_append(int count, int32_t *counter) {
    __shared__ int wsum[16];
    __shared__ int base;
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int incl = count;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int j = 0; j < nw; ++j) {
        const int t = wsum[j];
        before += j < wid ? t : 0;
        total += t;
    }
    if (threadIdx.x == 0) base = total > 0 ? atomicAdd(counter, total) : 0;
    __syncthreads();
    const int r = base + before + incl - count;
    __syncthreads();  // wsum and base are reused by the next call
    return r;
}

// Append the cells a lane's corrections touched to sweep s's touched list (every lane of the wave).
template <int W>
__device__ __forceinline__ void adj_append_touched(const AdjArgs &A, int s, const int32_t tsel[W + 1]) {
    int nt = 0;
#pragma unroll
    for (int k = 0; k <= W; ++k) nt += tsel[k] >= 0 ? 1 : 0;
    int b = wave_append(nt, &A.w.counters[kAdjT + s]);
    int32_t *T = A.w.tlist + (size_t)s * A.m.n_cells;
#pragma unroll
    for (int k = 0; k <= W; ++k)
        if (tsel[k] >= 0) T[b++] = tsel[k];
}

// per cell: start state of bounding (and phase A of its first sweep), lists, per-face adjoint
// buffers and phi_bar cleared
template <int W>
__global__ void __launch_bounds__(256) k_adj_prep(AdjArgs A) {
    const int n = A.m.n_cells;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t f = c; f < A.m.n_faces; f += (int64_t)gridDim.x * blockDim.x) A.phibar[f] = 0.0;
    bool offend = false;
    double x = 0.0;
    if (c < n) {
        x = A.raw[c];
        if (A.clip) {
            if (x < 0.0 && x >= -A.tol) x = 0.0;
            else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
        }
        A.w.x[c] = x;
        offend = x > 1.0 + A.tol || x < -A.tol;
        // with no sweep, the final clip makes a cell out of bounds (beyond round-off) a constant
        const bool clamped = A.n_iter == 0 && A.clip && offend && (x < -kRound || x > 1.0 + kRound);
        const double xb = clamped ? 0.0 : A.abar_new[c];
        A.w.xbar[c] = xb;
        A.w.pv[c] = raw_chopped(A.raw[c], A.clip, A.tol) ? 0.0 : xb / A.m.vol[c];
        A.w.cflag[c] = clamped ? 1 : 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int32_t v = A.m.slot_face[(size_t)k * n + c];
            if (v != kEmpty && v >= 0) {
                A.w.dVb[v] = 0.0;
                A.w.phib[v] = 0.0;
                A.w.dvcurbar[v] = 0.0;
            }
        }
    }
    if (A.n_iter < 1) return;  // uniform
    const int row = block_append(offend ? 1 : 0, &A.w.counters[kAdjL]);
    int32_t tsel[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) tsel[k] = -1;
    if (offend) {
        A.w.list[row] = c;
        adj_correct<W>(A, 0, c, row, x, A.w.cmark, tsel);
    }
    adj_append_touched<W>(A, 0, tsel);
}

// Phase B of sweep s: every touched cell applies its faces' corrections in ascending face order
// (round-off chop; clamp on the last sweep); a cell still out of bounds runs phase A of sweep s+1.
template <int W>
__global__ void __launch_bounds__(256) k_adj_sweep(AdjArgs A, int s) {
    const int n = A.m.n_cells, nf = A.m.n_faces;
    const DevMesh &m = A.m;
    const AdjWork &w = A.w;
    const int stride = gridDim.x * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    const bool last = s == A.n_iter - 1;
    if (s >= 1) {  // sweep s-1's corrections were read by the previous kernel: clear them
        const int np = w.counters[kAdjL + s - 1];
        double *stale = w.delta + (size_t)((s - 1) % 3) * nf;
        for (int i = t0; i < np; i += stride) {
            const int32_t P = w.list[(size_t)(s - 1) * n + i];
            const uint64_t flags = w.tflag[(size_t)(s - 1) * n + i];
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (flags & (kCorrBit << k)) {
                    const int32_t v = m.slot_pair[(size_t)P * W + k].x;
                    stale[v >= 0 ? v : ~v] = 0.0;
                }
        }
    }
    const double *delta = w.delta + (size_t)(s % 3) * nf;
    const int32_t *T = w.tlist + (size_t)s * n;
    int32_t *mark = w.cmark + (size_t)(s & 1) * n;
    int32_t *mark_next = w.cmark + (size_t)((s + 1) & 1) * n;
    const int nT = w.counters[kAdjT + s];
    const int nloop = (nT + 255) & ~255;  // whole work-groups iterate together
    for (int i0 = blockIdx.x * blockDim.x; i0 < nloop; i0 += stride) {
        const int i = i0 + threadIdx.x;
        bool again = false;
        int32_t Q = 0;
        double x = 0.0;
        if (i < nT) {
            Q = T[i];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int32_t vq = m.slot_pair[(size_t)Q * W + k].x;
                if (vq == kEmpty) continue;
                const double d = delta[vq >= 0 ? vq : ~vq];
                sum += vq >= 0 ? d : -d;
            }
            const double x0 = w.x[Q] - sum / m.vol[Q];
            x = x0;
            if (A.clip) {
                if (x < 0.0 && x >= -A.tol) x = 0.0;
                else if (x > 1.0 && x <= 1.0 + A.tol) x = 1.0;
                if (last) x = fmin(fmax(x, 0.0), 1.0);
            }
            if (fabs(x - x0) > kRound) w.cflag[Q] |= 1 << s;
            w.x[Q] = x;
            mark[Q] = 0;
            again = !last && (x > 1.0 + A.tol || x < -A.tol);
        }
        if (last) continue;  // uniform
        const int row = wave_append(again ? 1 : 0, &w.counters[kAdjL + s + 1]);
        int32_t tsel[W + 1];
#pragma unroll
        for (int k = 0; k <= W; ++k) tsel[k] = -1;
        if (again) {
            w.list[(size_t)(s + 1) * n + row] = Q;
            adj_correct<W>(A, s + 1, Q, row, x, mark_next, tsel);
        }
        adj_append_touched<W>(A, s + 1, tsel);
    }
}

// Reverse of sweep s, first half: the adjoint of each correction through the two cells it was
// applied to (a cell chopped or clamped in sweep s passes nothing back: it was a constant), and the
// chopped cells' adjoints zeroed.  The two sets are disjoint, so one kernel does both.  The forward
// replay is over: its face marks and this sweep's corrections are cleared here.
template <int W>
__global__ void __launch_bounds__(256) k_adj_unsweep_apply(AdjArgs A, int s) {
    const int n = A.m.n_cells, nf = A.m.n_faces;
    const DevMesh &m = A.m;
    const AdjWork &w = A.w;
    const int stride = gridDim.x * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = w.counters[kAdjL + s], nt = w.counters[kAdjT + s];
    const int32_t *L = w.list + (size_t)s * n;
    const int32_t *T = w.tlist + (size_t)s * n;
    double *delta = w.delta + (size_t)(s % 3) * nf;
    for (int i = t0; i < nl; i += stride) {
        const int32_t P = L[i];
        const uint64_t flags = w.tflag[(size_t)s * n + i];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (!(flags & (kCorrBit << k))) continue;
            const int2 q = m.slot_pair[(size_t)P * W + k];
            const int32_t v = q.x, o = q.y;
            const int32_t f = v >= 0 ? v : ~v;
            const double sP = v >= 0 ? 1.0 : -1.0;
            double db = 0.0;
            if (!(w.cflag[P] & (1 << s))) db -= sP * w.xbar[P] / m.vol[P];
            if (o >= 0 && !(w.cflag[o] & (1 << s))) db += sP * w.xbar[o] / m.vol[o];
            w.deltabar[f] = db;
            w.touched[f] = 0;
            delta[f] = 0.0;
        }
    }
    for (int j = t0; j < nt; j += stride) {
        const int32_t Q = T[j];
        if (w.cflag[Q] & (1 << s)) {
            w.xbar[Q] = 0.0;
            w.pv[Q] = 0.0;
        }
    }
}

// Reverse of sweep s, second half: through the corrections of each listed cell, to its bounding
// state, its outflow faces' fluxes and their dV (before bounding, or running from an earlier sweep).
template <int W>
__global__ void __launch_bounds__(256) k_adj_unsweep_correct(AdjArgs A, int s) {
    constexpr int R = 4 + 2 * W;
    const int n = A.m.n_cells;
    const DevMesh &m = A.m;
    const AdjWork &w = A.w;
    const int stride = gridDim.x * blockDim.x;
    const int nl = w.counters[kAdjL + s];
    const int32_t *L = w.list + (size_t)s * n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride) {
        const int32_t P = L[i];
        const uint64_t flags = w.tflag[(size_t)s * n + i];
        const double *rec = w.tape + ((size_t)s * n + i) * R;
        const bool over = flags & 1;
        const double sumcap = rec[2], r = rec[3];
        const double dtc = cell_dt(m, A.dt_dom, A.dt, P);
        double capb[W], dvnb[W];
        double rb = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            capb[k] = 0.0;
            dvnb[k] = 0.0;
            if (!(flags & (kCorrBit << k))) continue;
            const int32_t v = m.slot_pair[(size_t)P * W + k].x;
            const int32_t f = v >= 0 ? v : ~v;
            const double s_ = v >= 0 ? 1.0 : -1.0;
            const double ddb = w.deltabar[f] + w.dvcurbar[f];
            const double d_b = over ? s_ * ddb : -s_ * ddb;
            capb[k] = d_b * r;
            rb += d_b * rec[4 + k];
            dvnb[k] = w.dvcurbar[f];  // dvcur after = dV-now + correction
        }
        double needb = 0.0, sumcapb = 0.0;
        if ((flags & 4) && !(flags & 2)) {
            needb = rb / sumcap;
            sumcapb = -rb * r / sumcap;
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const double capk = rec[4 + k];
            if (!(capk > 0.0) || !(flags & 4)) continue;
            const int32_t v = m.slot_pair[(size_t)P * W + k].x;
            const int32_t f = v >= 0 ? v : ~v;
            const double s_ = v >= 0 ? 1.0 : -1.0;
            const double cb = capb[k] + sumcapb;
            const double outvb = over ? -cb : cb;
            if (over) w.phib[f] += cb * s_ * dtc;
            dvnb[k] += s_ * outvb;
            if (flags & (kTouchedBit << k)) {
                w.dvcurbar[f] = dvnb[k];
            } else {
                w.dVb[f] += dvnb[k];
                w.dvcurbar[f] = 0.0;
            }
        }
        const double xb = w.xbar[P] + needb * (over ? m.vol[P] : -m.vol[P]);
        w.xbar[P] = xb;
        w.pv[P] = raw_chopped(A.raw[P], A.clip, A.tol) ? 0.0 : xb / m.vol[P];
    }
}

// per cell: transposes of the update (through the round-off chop) and of the bulk fluxes
template <int W>
__device__ __forceinline__ void adj_faces_cell(const AdjArgs &A, int c) {
    const int n = A.m.n_cells;
    const DevMesh &m = A.m;
    // adjoint of the update before its round-off chop, and the same over the volume (kept per cell
    // by the kernels that change it, so a neighbour costs one load)
    const double bc = raw_chopped(A.raw[c], A.clip, A.tol) ? 0.0 : A.w.xbar[c];
    const double Vc = m.vol[c];
    const bool recon = A.kind[c] == 1;
    const double dtc = cell_dt(m, A.dt_dom, A.dt, c);
    double acc = bc;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int32_t v = m.slot_face[(size_t)k * n + c];
        if (v == kEmpty) continue;
        const int32_t f = v >= 0 ? v : ~v;
        const int32_t o = m.slot_nbr[(size_t)k * n + c];
        const double ph = A.phi[f];
        // alpha_raw(owner) -= dV/V_owner, alpha_raw(neighbour) += dV/V_neighbour
        double dvb;
        if (v >= 0) dvb = -bc / Vc + (o >= 0 ? A.w.pv[o] : 0.0);
        else dvb = -(o >= 0 ? A.w.pv[o] : 0.0) + bc / Vc;
        dvb += A.w.dVb[f];
        const double out = v >= 0 ? ph : -ph;
        if (out > 0.0) {
            if (recon) A.w.vbar[f] = dvb * ph;  // dV = phi * (swept integral of the interface cell)
            else acc += dvb * ph * dtc;         // dV = alpha_c phi dt
        }
        if (v >= 0) A.phibar[f] = (ph != 0.0 ? dvb * (A.dV0[f] / ph) : 0.0) + A.w.phib[f];
    }
    A.abar[c] = acc;
}

// per cell: transposes of the update and the bulk fluxes; the interface cells' work list
template <int W>
__global__ void __launch_bounds__(256) k_adj_faces(AdjArgs A) {
    const int n = A.m.n_cells;
    const int c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;  // contiguous ranges per XCD
    if (c < n) adj_faces_cell<W>(A, c);
    // the interface-cell directions k_adj_surface differentiates along: the isovalue, and each vertex
    // value that moves a cut point (a vertex no cut edge touches moves nothing: its rates are zero)
    uint32_t need = 0;
    int nbig = 0;  // a general polyhedron: every point value and the isovalue (kBigIsoDir)
    const bool big = c < n && A.m.cbig && A.m.cbig[c] >= 0;
    if (big && A.kind[c] == 1) {
        const int bi = A.m.cbig[c];
        nbig = A.m.bv_ptr[bi + 1] - A.m.bv_ptr[bi] + 1;
    } else if (c < n && A.kind[c] == 1) {
        const double iso = A.iso[c];
        uint32_t wet = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) wet |= (A.vert_alpha[8 * (size_t)c + v] > iso ? 1u : 0u) << v;
        if (A.m.cloop) {  // the edges of the cell's own face loops (a triangle's repeated point: none)
            for (int k = 0; k < 6; ++k) {
                const int32_t L = A.m.cloop[6 * (size_t)c + k];
                if (!((L >> 12) & 1)) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int p = (L >> (3 * i)) & 7, q = (L >> (3 * ((i + 1) & 3))) & 7;
                    if (((wet >> p) ^ (wet >> q)) & 1u) need |= (1u << p) | (1u << q);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 12; ++t)
                if (((wet >> kEdge[t][0]) ^ (wet >> kEdge[t][1])) & 1u)
                    need |= (1u << kEdge[t][0]) | (1u << kEdge[t][1]);
        }
        double *gb = A.w.gbuf + (size_t)kAdjG * c;
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (!((need >> v) & 1u)) {
                gb[v] = 0.0;
                gb[9 + v] = 0.0;
            }
        need |= 1u << 8;
    }
    int b = block_append(__popc(need), &A.w.counters[kAdjDirs]);
    for (int d = 0; d < 9; ++d)
        if ((need >> d) & 1u) A.w.dlist[b++] = ((int64_t)c << 4) | d;
    if (!A.m.cbig) return;  // uniform: no polyhedra in this mesh
    int bb = block_append(nbig, &A.w.counters[kAdjDirsBig]);
    for (int d = 0; d + 1 < nbig; ++d) A.w.dlist_big[bb++] = ((int64_t)c << 6) | d;
    if (nbig) A.w.dlist_big[bb] = ((int64_t)c << 6) | kBigIsoDir;
}

// interface cells: rates of the sub-volume and the swept integrals along each listed direction
__global__ void __launch_bounds__(256, 2) k_adj_surface(AdjArgs A) {
    const DevMesh &m = A.m;
    const int lv = threadIdx.x & (kLanes - 1);
    const int ngrp = (gridDim.x * blockDim.x) / kLanes;
    const int npair = A.w.counters[kAdjDirs];
    int fv[4];
    int fwd = lane_face_loop(lv, fv);
    bool face_on = lv < 6;
    for (int g = (blockIdx.x * blockDim.x + threadIdx.x) / kLanes; g < npair; g += ngrp) {
        const int64_t pr = A.w.dlist[g];
        const int c = (int)(pr >> 4);
        const int dir = (int)(pr & 15);  // 0..7: vertex value dir, 8: the isovalue
        if (m.cloop) {  // cells other than hexahedra: the cell's own face loops, as in the step
            const int32_t L = lv < 6 ? m.cloop[6 * (size_t)c + lv] : 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) fv[i] = (L >> (3 * i)) & 7;
            fwd = (L >> 16) & 15;
            face_on = (L >> 12) & 1;
        }
        const double aP = A.alpha[c];
        const double V6 = 6.0 * m.vol[c];
        const double dtc = cell_dt(m, A.dt_dom, A.dt, c);
        const double *cx = m.cxyz + 24 * (size_t)c + 3 * lv;
        D3 xv{cx[0], cx[1], cx[2]};
        const double av = A.vert_alpha[8 * (size_t)c + lv];
        const D3 xm = 0.125 * grp_sum3(xv);
        xv = xv - xm;
        DFace f;
        f.active = face_on;
        f.planar = (m.cflags[c] >> min(lv, 5)) & 1;
        f.fwd = fwd;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f.q[i] = D3{grp_get(xv.x, fv[i]), grp_get(xv.y, fv[i]), grp_get(xv.z, fv[i])};
            f.aq[i] = Dl{grp_get(av, fv[i]), fv[i] == dir ? 1.0 : 0.0};
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const Dl d = ((fwd >> i) & 1) ? f.aq[(i + 1) & 3] - f.aq[i] : f.aq[i] - f.aq[(i + 1) & 3];
            f.inv[i] = d.v != 0.0 ? dinv(d) : dc(0.0);
        }
        const double iso = A.iso[c];
        // one pass along this direction: the sub-volume's rate (at fixed isovalue for a vertex
        // value, along the isovalue for direction 8), and the isoface and swept integrals
        const Dl isod{iso, dir == 8 ? 1.0 : 0.0};
        DV3 o, cseg;
        const Dl g0 = dcell_vsub6(f, isod, &o, &cseg);
        const Dl nrm = dnorm(cseg);
        double contrib = 0.0;
        if (nrm.v > 0.0) {
            const DV3 nS = dinv(nrm) * cseg;
            DV3 acc;
            Dl ws;
            dface_centre_part(f, isod, o, nS, acc, ws);
            acc = dgrp_sum3(acc);
            ws = dgrp_sum(ws);
            const DV3 xS = dinv(3.0 * ws) * acc;
            const Dl un = A.U[c] * nS.x + A.U[m.n_cells + c] * nS.y + A.U[2 * (size_t)m.n_cells + c] * nS.z;
            if (f.active) {
                const int32_t v = m.lface[6 * (size_t)c + lv];
                if (v != kEmpty) {
                    const int32_t fid = v >= 0 ? v : ~v;
                    const double ph = A.phi[fid];
                    const double out = v >= 0 ? ph : -ph;
                    if (out > 0.0) {
                        Dl dq[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) dq[i] = ddot(dv(f.q[i]) - xS, nS);
                        Dl accI = dc(0.0);
                        double Af = 0.0;
                        if (f.planar) {
                            const double A1 = 0.5 * norm3(cross(f.q[1] - f.q[0], f.q[2] - f.q[0]));
                            const double A2 = 0.5 * norm3(cross(f.q[2] - f.q[0], f.q[3] - f.q[0]));
                            accI = A1 * dtri_sweep(dq[0], dq[1], dq[2], un, dtc) + A2 * dtri_sweep(dq[0], dq[2], dq[3], un, dtc);
                            Af = A1 + A2;
                        } else {
                            const D3 ap = 0.25 * (f.q[0] + f.q[1] + f.q[2] + f.q[3]);
                            const Dl dap = ddot(dv(ap) - xS, nS);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const double Ai = 0.5 * norm3(cross(f.q[i] - ap, f.q[(i + 1) & 3] - ap));
                                accI = accI + Ai * dtri_sweep(dap, dq[i], dq[(i + 1) & 3], un, dtc);
                                Af += Ai;
                            }
                        }
                        contrib = A.w.vbar[fid] * (accI.d / Af);
                    }
                }
            }
        }
        // this direction's rate of six times the sub-volume and of the faces' adjoint-weighted swept
        // integrals; k_adj_points and k_adj_cells combine them (adj_vertex, adj_alpha)
        const double gsum = grp_sum(contrib);
        double *gb = A.w.gbuf + (size_t)kAdjG * c;
        if (lv == 0) {
            gb[dir] = g0.d;
            gb[9 + dir] = gsum;
        }
        if (dir == 8) {
            // at a jump of the sub-volume the isovalue is a vertex value and moves with it
            const bool jump = fabs(g0.v - aP * V6) > 1e-9 * V6;
            const uint64_t hit = __ballot(jump && av == iso);
            const int mvert = (int)((hit >> (__lane_id() & ~(kLanes - 1))) & 0xFF);
            if (lv == 0) {
                gb[18] = jump ? (double)(mvert ? __ffs(mvert) - 1 : -1) : -2.0;
                gb[19] = V6;
            }
        }
    }
}

// The isovalue moves with the volume constraint, so the adjoint of vertex value v is its rate at
// fixed isovalue plus the isovalue's rate along v times the rate along the isovalue: with G the
// rates of six times the sub-volume and C those of the adjoint-weighted swept integrals,
// iso' = -G_v / G_iso, and alpha_P's is iso' = V6 / G_iso times C_iso.  At a jump the isovalue is
// the jumping vertex's value (iso' = 1 for it, 0 otherwise, and 0 for alpha_P).
__device__ __forceinline__ double adj_vertex(const double *gb, int v) {
    const double jump = gb[18], gx = gb[8];
    double xdot;
    if (jump > -2.0) xdot = (double)v == jump ? 1.0 : 0.0;
    else xdot = gx != 0.0 ? -gb[v] / gx : 0.0;
    return gb[9 + v] + xdot * gb[17];
}
__device__ __forceinline__ double adj_alpha(const double *gb) {
    const double gx = gb[8];
    const double xdot = gb[18] > -2.0 ? 0.0 : (gx != 0.0 ? gb[19] / gx : 0.0);
    return xdot * gb[17];
}

// ------------------------------------------------------------------ general polyhedra (16 lanes)
// One group of sixteen lanes per (polyhedron, direction), lane lf on the cell's face lf, as in the
// forward polyhedron kernel: the cell's points (relative to their mean) and vertex values sit in
// LDS, the vertex values recomputed through the same stencils in the same order, so they are the
// forward's bits.  Directions 0 .. nv-1 are the points' values, kBigIsoDir the isovalue; the rates
// are stored per polyhedron: G (six times the sub-volume) at [0, kBigIsoDir], C (the faces'
// adjoint-weighted swept integrals) at kBigC + [0, kBigIsoDir], then the jump and 6V.

struct BPt {
    double x, y, z, a;
};
__device__ __forceinline__ double a16(double v) {  // the 8-lane butterfly, then the row's halves
    v = grp_sum(v);
    return v + dpp_move<0x140>(v);
}
__device__ __forceinline__ Dl da16(Dl a) { return {a16(a.v), a16(a.d)}; }
__device__ __forceinline__ DV3 da16_3(DV3 a) { return {da16(a.x), da16(a.y), da16(a.z)}; }
__device__ __forceinline__ void adj_grp_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kBGrp * kBGrpPerBlock) k_adj_surface_big(AdjArgs A) {
    __shared__ BPt spt[kBGrpPerBlock][kBPts];
    const DevMesh &m = A.m;
    const int g = threadIdx.x / kBGrp, lf = threadIdx.x % kBGrp;
    BPt *P = spt[g];
    const int npair = A.w.counters[kAdjDirsBig];
    const size_t nc = m.n_cells;
    const DV3 Z = dv(D3{0, 0, 0});
    for (int idx = blockIdx.x * kBGrpPerBlock + g; idx < npair; idx += gridDim.x * kBGrpPerBlock) {
        const int64_t pr = A.w.dlist_big[idx];
        const int c = (int)(pr >> 6), dir = (int)(pr & 63);
        const int bi = m.cbig[c];
        const double aP = A.alpha[c];
        const double V6 = 6.0 * m.vol[c];
        const double dtc = cell_dt(m, A.dt_dom, A.dt, c);
        const int v0 = m.bv_ptr[bi], nv = m.bv_ptr[bi + 1] - v0;
        D3 xp[2];
        double ap[2];
        D3 xs{0, 0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lf + kBGrp * h;
            xp[h] = D3{0, 0, 0};
            ap[h] = 0.0;
            if (i < nv) {
                const double *q = m.bv_xyz + 3 * (size_t)(v0 + i);
                xp[h] = D3{q[0], q[1], q[2]};
                const int k = m.bv_cls[v0 + i];
                double av = 0.0;
                for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e) av += m.st_w[e] * A.alpha[m.st_cell[e]];
                ap[h] = av;
                xs = xs + xp[h];
            }
        }
        const D3 xm = (1.0 / nv) * D3{a16(xs.x), a16(xs.y), a16(xs.z)};
        adj_grp_sync();  // the previous pair's reads of P are done
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lf + kBGrp * h;
            if (i < nv) P[i] = BPt{xp[h].x - xm.x, xp[h].y - xm.y, xp[h].z - xm.z, ap[h]};
        }
        adj_grp_sync();
        const double iso = A.iso[c];
        const Dl isod{iso, dir == kBigIsoDir ? 1.0 : 0.0};
        // this lane's face: its loop of local points (outward), planarity, flux face
        const int f0 = m.bf_ptr[bi], nf = m.bf_ptr[bi + 1] - f0;
        const bool face = lf < nf;
        const int lb = face ? m.bl_ptr[f0 + lf] : 0;
        const int ln = face ? m.bl_ptr[f0 + lf + 1] - lb : 0;
        const bool planar = face && m.bf_planar[f0 + lf];
        auto loc = [&](int pos) { return m.bl_vtx[lb + pos]; };
        auto dpt = [&](int l) { return DV3{dc(P[l].x), dc(P[l].y), dc(P[l].z)}; };
        auto dval = [&](int l) { return Dl{P[l].a, l == dir ? 1.0 : 0.0}; };
        // cut point of the edge between local points l1 and l2, exactly one of them wet: from the
        // wet end, as the forward computes it
        auto cut = [&](int l1, int l2, bool w1) {
            const int lw = w1 ? l1 : l2, ld = w1 ? l2 : l1;
            const Dl lam = (isod - dval(lw)) / (dval(ld) - dval(lw));
            return dpt(lw) + lam * (dpt(ld) - dpt(lw));
        };
        // the face's share of six times the sub-volume and of the isoface sums (wet iff a > iso)
        DV3 C = Z, pacc = Z, psum = Z, lastexit = Z, first_entry = Z, cseg = Z, oacc = Z;
        Dl pl = dc(0.0), oL = dc(0.0);
        int cnt = 0;
        bool have_exit = false, pend = false;
        auto iso_edge = [&](DV3 s0, DV3 s1) {
            const Dl l = dnorm(s1 - s0);
            cseg = cseg + dcross(s0, s1);
            oacc = oacc + (0.5 * l) * (s0 + s1);
            oL = oL + l;
        };
        for (int i = 0; i < ln; ++i) {
            const int li = loc(i), lj = loc(i + 1 < ln ? i + 1 : 0);
            const bool wi = P[li].a > iso, wj = P[lj].a > iso;
            const DV3 xi = dpt(li), xj = dpt(lj);
            DV3 ct = Z;
            if (wi != wj) ct = cut(li, lj, wi);
            if (!wi && wj) {
                if (have_exit) iso_edge(ct, lastexit);
                else { pend = true; first_entry = ct; }
            }
            if (wi && !wj) { lastexit = ct; have_exit = true; }
            if (wi || wj) {
                const DV3 u = wi ? xi : ct, v = wj ? xj : ct;
                C = C + dcross(u, v);
                const Dl l = dnorm(v - u);
                pacc = pacc + (0.5 * l) * (u + v);
                pl = pl + l;
            }
            if (wi) psum = psum + xi;
            if (wi != wj) psum = psum + ct;
            cnt += (wi ? 1 : 0) + (wi != wj ? 1 : 0);
        }
        if (pend) iso_edge(first_entry, lastexit);
        C = C - cseg;  // the isoface edges close the wet loop, walked exit to entry
        Dl v6 = dc(0.0);
        if (cnt >= 3) {
            DV3 apx = dpt(loc(0));
            if (!planar) {
                const DV3 tot = pacc + oacc;
                const Dl tl = pl + oL;
                apx = tl.v > 0.0 ? dinv(tl) * tot : (1.0 / cnt) * psum;
            }
            v6 = ddot(apx, C);
        }
        const DV3 gcseg = da16_3(cseg), goacc = da16_3(oacc);
        const Dl goL = da16(oL);
        const DV3 o = goL.v > 0.0 ? dinv(goL) * goacc : Z;
        const Dl g0 = da16(v6) + ddot(o, gcseg);
        const Dl nrm = dnorm(gcseg);
        double contrib = 0.0;
        if (nrm.v > 0.0) {
            const DV3 nS = dinv(nrm) * gcseg;
            // the isoface centre: fan triangles (o, entry, preceding exit) weighted along n_S
            DV3 acc = Z;
            Dl ws = dc(0.0);
            DV3 le = Z, fe = Z;
            bool hx = false, pd = false;
            auto tri = [&](DV3 s0, DV3 s1) {
                const Dl wt = ddot(dcross(s0 - o, s1 - o), nS);
                acc = acc + wt * (o + s0 + s1);
                ws = ws + wt;
            };
            for (int i = 0; i < ln; ++i) {
                const int li = loc(i), lj = loc(i + 1 < ln ? i + 1 : 0);
                const bool wi = P[li].a > iso, wj = P[lj].a > iso;
                if (!wi && wj) {
                    const DV3 ct = cut(li, lj, false);
                    if (hx) tri(ct, le);
                    else { pd = true; fe = ct; }
                }
                if (wi && !wj) { le = cut(li, lj, true); hx = true; }
            }
            if (pd) tri(fe, le);
            acc = da16_3(acc);
            ws = da16(ws);
            const DV3 xS = dinv(3.0 * ws) * acc;
            const Dl un = A.U[c] * nS.x + A.U[nc + c] * nS.y + A.U[2 * nc + c] * nS.z;
            if (face) {
                const int32_t v = m.bf_face[f0 + lf];
                if (v != kEmpty) {
                    const int32_t fid = v >= 0 ? v : ~v;
                    const double ph = A.phi[fid];
                    const double out = v >= 0 ? ph : -ph;
                    if (out > 0.0) {
                        // the face fanned about its vertex mean, each triangle's swept fraction
                        D3 fm{0, 0, 0};
                        for (int i = 0; i < ln; ++i) {
                            const int l = loc(i);
                            fm = fm + D3{P[l].x, P[l].y, P[l].z};
                        }
                        fm = (1.0 / ln) * fm;
                        const Dl dap = ddot(dv(fm) - xS, nS);
                        Dl accI = dc(0.0);
                        double Af = 0.0;
                        for (int i = 0; i < ln; ++i) {
                            const int li = loc(i), lj = loc(i + 1 < ln ? i + 1 : 0);
                            const D3 xi{P[li].x, P[li].y, P[li].z}, xj{P[lj].x, P[lj].y, P[lj].z};
                            const double Ai = 0.5 * norm3(cross(xi - fm, xj - fm));
                            accI = accI + Ai * dtri_sweep(dap, ddot(dv(xi) - xS, nS), ddot(dv(xj) - xS, nS), un, dtc);
                            Af += Ai;
                        }
                        contrib = A.w.vbar[fid] * (accI.d / Af);
                    }
                }
            }
        }
        const double gsum = a16(contrib);
        double *gb = A.w.gbig + (size_t)kAdjGBig * bi;
        const int slot = dir == kBigIsoDir ? kBigIsoDir : dir;
        if (lf == 0) {
            gb[slot] = g0.d;
            gb[kBigC + slot] = gsum;
        }
        if (dir == kBigIsoDir) {
            // at a jump of the sub-volume the isovalue is a vertex value and moves with it: the
            // lowest point at the isovalue
            const bool jump = fabs(g0.v - aP * V6) > 1e-9 * V6;
            const int base = __lane_id() & ~(kBGrp - 1);
            const uint32_t lo = (uint32_t)(__ballot(lf < nv && P[lf].a == iso) >> base) & 0xFFFFu;
            const uint32_t hi = (uint32_t)(__ballot(lf + kBGrp < nv && P[lf + kBGrp].a == iso) >> base) & 0xFFFFu;
            const uint32_t at = lo | (hi << 16);
            if (lf == 0) {
                gb[kBigJump] = jump ? (double)(at ? __ffs((int)at) - 1 : -1) : -2.0;
                gb[kBigV6] = V6;
            }
        }
        // zero rates for the unused point slots, so that the gathers may read any of them
        if (dir == kBigIsoDir && lf == 0)
            for (int v = nv; v < kBigIsoDir; ++v) gb[v] = gb[kBigC + v] = 0.0;
    }
}

__device__ __forceinline__ double adj_vertex_big(const double *gb, int v) {
    const double jump = gb[kBigJump], gx = gb[kBigIsoDir];
    double xdot;
    if (jump > -2.0) xdot = (double)v == jump ? 1.0 : 0.0;
    else xdot = gx != 0.0 ? -gb[v] / gx : 0.0;
    return gb[kBigC + v] + xdot * gb[kBigC + kBigIsoDir];
}
__device__ __forceinline__ double adj_alpha_big(const double *gb) {
    const double gx = gb[kBigIsoDir];
    const double xdot = gb[kBigJump] > -2.0 ? 0.0 : (gx != 0.0 ? gb[kBigV6] / gx : 0.0);
    return xdot * gb[kBigC + kBigIsoDir];
}

// Transpose of the vertex interpolation, as two gathers in a fixed order (no atomics, so the
// gradient is the same bits on every run): each point class sums the vertex adjoints of the
// reconstructed cells that share it, then each cell adds its classes' sums times its weight in
// their stencils.  A cell that shares a class twice (two of its vertices are periodic images of
// one point) appears twice in the class's stencil, with one weight per image; its vertices are
// summed at its first entry and each of its distinct classes is taken once.
__global__ void __launch_bounds__(256) k_adj_points(AdjArgs A) {
    const DevMesh &m = A.m;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m.n_classes) return;
    const int e0 = m.st_ptr[k], e1 = m.st_ptr[k + 1];
    double sum = 0.0;
    // stencil entries eight at a time, their cells' kinds all in flight together; most classes
    // have no reconstructed cell, and those skip the rest
    for (int eb = e0; eb < e1; eb += 8) {
        int32_t sc[8], kd[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) sc[j] = eb + j < e1 ? m.st_cell[eb + j] : -1;
#pragma unroll
        for (int j = 0; j < 8; ++j) kd[j] = sc[j] >= 0 ? A.kind[sc[j]] : 0;
        for (int j = 0; j < 8; ++j) {
            if (kd[j] != 1) continue;
            const int32_t c = sc[j];
            bool first = true;
            for (int e2 = e0; e2 < eb + j; ++e2) first = first && m.st_cell[e2] != c;
            if (!first) continue;
            if (m.cbig && m.cbig[c] >= 0) {
                const int bi = m.cbig[c], v0 = m.bv_ptr[bi], nv = m.bv_ptr[bi + 1] - v0;
                for (int v = 0; v < nv; ++v)
                    if (m.bv_cls[v0 + v] == k) sum += adj_vertex_big(A.w.gbig + (size_t)kAdjGBig * bi, v);
                continue;
            }
#pragma unroll
            for (int v = 0; v < 8; ++v)
                if (m.cpt[8 * (size_t)c + v] == k) sum += adj_vertex(A.w.gbuf + (size_t)kAdjG * c, v);
        }
    }
    A.w.pbar[k] = sum;
}

__global__ void __launch_bounds__(256) k_adj_cells(AdjArgs A) {
    const DevMesh &m = A.m;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    // nothing reads the counters after the surface kernels: leave them zero for the next call
    if (blockIdx.x == 0 && threadIdx.x < kAdjNum) A.w.counters[threadIdx.x] = 0;
    if (c >= m.n_cells) return;
    double acc = A.abar[c];
    if (m.cbig && m.cbig[c] >= 0) {
        // a general polyhedron: the distinct classes of all its points
        const int bi = m.cbig[c], v0 = m.bv_ptr[bi], nv = m.bv_ptr[bi + 1] - v0;
        if (A.kind[c] == 1) acc += adj_alpha_big(A.w.gbig + (size_t)kAdjGBig * bi);
        for (int v = 0; v < nv; ++v) {
            const int32_t k = m.bv_cls[v0 + v];
            bool seen = false;
            for (int u = 0; u < v; ++u) seen = seen || m.bv_cls[v0 + u] == k;
            const double pbk = A.w.pbar[k];
            if (seen || pbk == 0.0) continue;
            for (int e = m.st_ptr[k]; e < m.st_ptr[k + 1]; ++e)
                if (m.st_cell[e] == c) acc += m.st_w[e] * pbk;
        }
        A.abar[c] = acc;
        return;
    }
    if (A.kind[c] == 1) acc += adj_alpha(A.w.gbuf + (size_t)kAdjG * c);
    int32_t cls[8];
    double pb[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) cls[v] = m.cpt[8 * (size_t)c + v];
#pragma unroll
    for (int v = 0; v < 8; ++v) pb[v] = A.w.pbar[cls[v]];  // all eight in flight together
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        bool seen = false;
#pragma unroll
        for (int u = 0; u < v; ++u) seen = seen || cls[u] == cls[v];
        if (seen || pb[v] == 0.0) continue;
        for (int e = m.st_ptr[cls[v]]; e < m.st_ptr[cls[v] + 1]; ++e)
            if (m.st_cell[e] == c) acc += m.st_w[e] * pb[v];
    }
    A.abar[c] = acc;
}


template <int W>
hipError_t launch_adj_w(const AdjArgs &a, hipStream_t s) {
    static_assert(W <= 16, "the bounding tape's flags hold 16 slots");
    const int n = a.m.n_cells;
    const int g = (n + 255) / 256;
    const int gb = std::max(1, std::min(g, (int)kAdjBoundBlocks));
    hipLaunchKernelGGL(k_adj_prep<W>, dim3(g), dim3(256), 0, s, a);
    for (int it = 0; it < a.n_iter; ++it) hipLaunchKernelGGL(k_adj_sweep<W>, dim3(gb), dim3(256), 0, s, a, it);
    for (int it = a.n_iter - 1; it >= 0; --it) {
        hipLaunchKernelGGL(k_adj_unsweep_apply<W>, dim3(gb), dim3(256), 0, s, a, it);
        hipLaunchKernelGGL(k_adj_unsweep_correct<W>, dim3(gb), dim3(256), 0, s, a, it);
    }
    hipLaunchKernelGGL(k_adj_faces<W>, dim3(g), dim3(256), 0, s, a);
    const int gs = std::max(1, std::min(2048, (int)((9L * n * kLanes + 255) / 256)));
    hipLaunchKernelGGL(k_adj_surface, dim3(gs), dim3(256), 0, s, a);
    if (a.m.cbig) {
        const int gb = std::max(1, std::min(1024, (int)((33L * a.w.big_cap + kBGrpPerBlock - 1) / kBGrpPerBlock)));
        hipLaunchKernelGGL(k_adj_surface_big, dim3(gb), dim3(kBGrp * kBGrpPerBlock), 0, s, a);
    }
    hipLaunchKernelGGL(k_adj_points, dim3((a.m.n_classes + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_adj_cells, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(const DevMesh &m, const Params &p, const StepArgs &a, const AdjInputs &in, const AdjWork &w,
                          hipStream_t s) {
    if (p.n_bound_iter > kAdjMaxSweeps) return hipErrorInvalidValue;
    // phi_bar starts at zero in k_adj_prep (faces that carry no flux keep it); the counters are
    // zero from the workspace's allocation and left zero by k_adj_cells at the end of every call
    AdjArgs A{m, a.alpha, a.phi, a.U, a.dt, a.dt_dom, p.eps_surf, p.bound_tol, p.clip, p.n_bound_iter,
              in.vert_alpha, in.kind, in.iso, in.dV, in.raw, in.abar_new, in.abar, in.phibar, w};
    switch (m.W) {  // the slot widths of the step's update (polyhedra pad theirs to 8, 12 or 16)
        case 1: return launch_adj_w<1>(A, s);
        case 2: return launch_adj_w<2>(A, s);
        case 3: return launch_adj_w<3>(A, s);
        case 4: return launch_adj_w<4>(A, s);
        case 5: return launch_adj_w<5>(A, s);
        case 6: return launch_adj_w<6>(A, s);
        case 8: return launch_adj_w<8>(A, s);
        case 12: return launch_adj_w<12>(A, s);
        case 16: return launch_adj_w<16>(A, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace isoadv
