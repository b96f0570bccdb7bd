// Ghost-fluid face data after advection (Section 3.1, Eqs. 12-20).
//
// One thread per mesh face.  A face with a cell on each side (an internal face, or the face of a
// cyclic pair that carries the flux, whose far cell is seen through the pair's translation) lies
// on the free surface when its two cells sit on opposite sides of alpha = 1/2 (wet: alpha > 1/2,
// the heavy fluid).  There the kernel writes the interface position lambda (Eq. 13, from the
// face's owner), the jump H = p_d^- - p_d^+ = (rho^+ - rho^-) g . x_Gamma at x_Gamma (Eq. 12;
// the sign follows Eq. 3 with a continuous pressure and Eq. 7), the weighted inverse density
// beta_w (Eq. 18, with lambda measured from the heavy cell), and the ghost values: the heavy
// fluid's p_d extended to the dry cell (Eq. 20) and the light fluid's extended to the wet cell
// (the mirror of Eqs. 17-20).  Every other face gets lambda = -1, H = beta_w = 0 and the plain
// cell values (the owner's value on both sides where there is no second cell).
//
// The work is a gather of two cells' alpha and p_d per face and five streamed stores: bound by
// HBM bandwidth, and three quarters of the bytes are the stores.  Faces are numbered owner by
// owner, so consecutive threads touch neighbouring cells.  Work-groups are dealt to the XCDs in
// the hardware's round-robin order: giving each XCD a contiguous range of faces (which keeps a
// cell's lines behind one L2 for the faces of the cells above it) measured 8 % slower, the store
// streams being what counts; work-groups of 512 measured 3 % faster than 256 or 128.  FMA
// contraction is off: the arithmetic rounds operation by operation in the order written.
#include "device_common.h"
#include "internal.h"

namespace isoadv {

namespace {

typedef int32_t v2i __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(512) void k_gfm_faces(GfmArgs A) {
#pragma clang fp contract(off)
    const int64_t f = (int64_t)blockIdx.x * 512 + threadIdx.x;
    if (f >= A.n_faces) return;
    const v2i pn = __builtin_nontemporal_load(reinterpret_cast<const v2i *>(A.fcell) + f);
    const int32_t P = pn.x, N = pn.y;
    const double aP = A.alpha[P], pP = A.p_d[P];
    double lam = -1.0, H = 0.0, bw = 0.0, g_own = pP, g_nbr = pP;
    if (N >= 0) {
        const double aN = A.alpha[N], pN = A.p_d[N];
        g_nbr = pN;
        const bool wetP = aP > 0.5, wetN = aN > 0.5;
        if (wetP != wetN) {
            double xP[3], xN[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xP[d] = A.ccen[3 * (size_t)P + d];
                xN[d] = A.ccen[3 * (size_t)N + d];
            }
            if (f >= A.n_internal) {  // cyclic: the far cell's centre in the owner's frame
                const double *T = A.ptrans + 3 * A.bpatch[f - A.n_internal];
#pragma unroll
                for (int d = 0; d < 3; ++d) xN[d] -= T[d];
            }
            lam = (aP - 0.5) / (aP - aN);  // Eq. 13
            double xG[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) xG[d] = xP[d] + lam * (xN[d] - xP[d]);  // Eq. 12
            H = A.drho * (A.g[0] * xG[0] + A.g[1] * xG[1] + A.g[2] * xG[2]);
            const double lw = wetP ? lam : 1.0 - lam;  // distance fraction from the heavy cell
            bw = lw * A.b_light + (1.0 - lw) * A.b_heavy;  // Eq. 18
            const double pW = wetP ? pP : pN, pD = wetP ? pN : pP;
            const double cl = A.b_light / bw, ch = A.b_heavy / bw;
            const double to_dry = cl * pD + (1.0 - cl) * pW - cl * H;  // Eq. 20
            const double to_wet = ch * pW + (1.0 - ch) * pD + ch * H;  // its mirror
            g_nbr = wetP ? to_dry : to_wet;
            g_own = wetP ? to_wet : to_dry;
        }
    }
    __builtin_nontemporal_store(lam, A.lambda + f);
    __builtin_nontemporal_store(H, A.jump + f);
    __builtin_nontemporal_store(bw, A.beta_w + f);
    __builtin_nontemporal_store(g_own, A.ghost_own + f);
    __builtin_nontemporal_store(g_nbr, A.ghost_nbr + f);
}

}  // namespace

hipError_t launch_gfm_faces(const GfmArgs &a, hipStream_t s) {
    if (a.n_faces <= 0) return hipSuccess;
    const int blocks = (a.n_faces + 511) / 512;
    hipLaunchKernelGGL(k_gfm_faces, dim3(blocks), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace isoadv
