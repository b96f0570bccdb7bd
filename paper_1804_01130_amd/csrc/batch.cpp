// Ensembles of independent meshes advanced together.  The members' device arrays are
// concatenated into one mesh (indices offset, cells of member d in [dom_off[d], dom_off[d+1])),
// so each kernel of a step is one launch over every member; a whole multi-step run is captured
// once as a HIP graph and replayed.  Each member's cells read its own time step from a device
// table, so every member computes bit for bit what its own plan computes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

using namespace isoadv;

namespace {
constexpr int32_t kMaxGraphSteps = 256;  // longer runs are launched step by step
}

struct iso_batch {
    iso_mesh *u = nullptr;     // the union mesh (device arrays only)
    iso_plan *plan = nullptr;  // options and workspace over the union
    int32_t n = 0;
    std::vector<int64_t> cell_off, face_off;
    double *dt_dev = nullptr;   // [n]
    double *dt_host = nullptr;  // pinned [n]
    double *tmp = nullptr;      // [N] second state buffer
    double *scratch = nullptr;  // [N] state copy for tuning trials
    hipStream_t user = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    LaunchCfg cfg{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        const double *alpha = nullptr, *phi = nullptr, *U = nullptr;
        int64_t ps = 0, us = 0;
        int32_t steps = 0;
        LaunchCfg cfg{};
    } key;
    bool have_graph = false;
};

namespace {

bool same_cfg(const LaunchCfg &a, const LaunchCfg &b) {
    return a.block_cells == b.block_cells && a.surface_blocks == b.surface_blocks &&
           a.surface_waves == b.surface_waves && a.bound_blocks == b.bound_blocks &&
           a.compact_slots == b.compact_slots;
}

void drop_graph(iso_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->have_graph = false;
}

template <class T>
bool dev_alloc(iso_mesh *u, T **p, int64_t count) {
    const size_t bytes = std::max<size_t>(1, (size_t)count) * sizeof(T);
    if (hipMalloc((void **)p, bytes) != hipSuccess) return false;
    u->allocations.push_back(*p);
    u->device_bytes += (int64_t)bytes;
    return true;
}

// steps [0, n_steps) of the ensemble from state alpha (alternating with b->tmp), ending in alpha
hipError_t enqueue_steps(iso_batch *b, double *alpha, const double *phi, int64_t ps, const double *U, int64_t us,
                         int32_t n_steps, const LaunchCfg &cfg) {
    const Params prm = step_params(b->plan->opt);
    for (int32_t s = 0; s < n_steps; ++s) {
        double *in = (s & 1) ? b->tmp : alpha;
        double *outp = (s & 1) ? alpha : b->tmp;
        StepArgs a{in, phi + (size_t)s * ps, U + (size_t)s * us, outp, 0.0, b->dt_dev};
        hipError_t e = launch_step(b->u->dev, b->plan->work, prm, a, nullptr, cfg, false, b->stream, nullptr);
        if (e != hipSuccess) return e;
    }
    if (n_steps & 1) return launch_copy_f64(b->tmp, alpha, b->u->n_cells, b->stream);
    return hipSuccess;
}

iso_status upload_dt(iso_batch *b, const double *dt) {
    for (int32_t i = 0; i < b->n; ++i)
        if (!(dt[i] > 0) || !std::isfinite(dt[i])) return fail(ISO_EINVAL, "dt must be positive and finite");
    // the pinned staging buffer may still feed an earlier copy
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(ISO_EDEVICE, "stream sync failed");
    std::memcpy(b->dt_host, dt, sizeof(double) * b->n);
    if (hipMemcpyAsync(b->dt_dev, b->dt_host, sizeof(double) * b->n, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return fail(ISO_EDEVICE, "dt upload failed");
    return ISO_OK;
}

std::string signature(const iso_batch *b) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the member layout
    auto mix = [&](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (int64_t v : b->cell_off) mix(v);
    for (int64_t v : b->face_off) mix(v);
    char buf[96];
    std::snprintf(buf, sizeof(buf), "n%d_c%lld_f%lld_%016llx", b->n, (long long)b->cell_off.back(),
                  (long long)b->face_off.back(), (unsigned long long)h);
    return buf;
}

}  // namespace

extern "C" {

void iso_batch_destroy(iso_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->plan) iso_plan_destroy(b->plan);
    if (b->u) iso_mesh_destroy(b->u);
    if (b->dt_host) (void)hipHostFree(b->dt_host);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

iso_status iso_batch_create(const iso_mesh *const *meshes, int32_t n, const iso_options *opt, void *hip_stream,
                            iso_batch **out) {
    if (!out) return fail(ISO_EINVAL, "out is null");
    *out = nullptr;
    if (!meshes || n < 1) return fail(ISO_EINVAL, "an ensemble needs at least one mesh");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ISO_EDEVICE, "no HIP device");
    int64_t N = 0, F = 0, K = 0, S = 0, P = 0, NF = 0;
    int64_t NB = 0, NBV = 0, NBF = 0, NBL = 0;  // general polyhedra: cells, points, faces, loop entries
    int32_t W = 1, big_face_pts = 0;
    bool generic = false, any_big = false, all_big = true, narrow = false, wide = false;
    for (int32_t i = 0; i < n; ++i) {
        const iso_mesh *m = meshes[i];
        if (!m) return fail(ISO_EINVAL, "null mesh in the ensemble");
        if (m->device != dev) return fail(ISO_EINVAL, "ensemble members must live on the current device");
        generic = generic || m->generic;
        if (m->dev.cbig) {
            any_big = true;
            big_face_pts = std::max(big_face_pts, m->dev.big_face_pts);
            (m->dev.big_face_pts > 4 ? wide : narrow) = true;
            NB += m->n_big; NBV += m->n_bv; NBF += m->n_bf; NBL += m->n_bl;
        }
        all_big = all_big && m->dev.all_big;
        N += m->n_cells; F += m->n_faces; K += m->n_classes; S += m->st_nnz; P += m->dev.n_patches;
        NF += m->n_flux;
        W = std::max(W, m->W);
    }
    const int64_t lim = std::numeric_limits<int32_t>::max() - 1;
    if (N > lim || F > lim || K > lim || S > lim || P > lim || 3 * NBV > lim || NBF > lim || NBL > lim ||
        24 * N > (int64_t)1 << 62)
        return fail(ISO_EINVAL, "ensemble too large for 32-bit indices");
    all_big = all_big && any_big;

    iso_batch *b = new iso_batch();
    b->n = n;
    b->user = static_cast<hipStream_t>(hip_stream);
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        iso_batch_destroy(b);
        return fail(ISO_EDEVICE, "stream or event creation failed");
    }
    iso_mesh *u = new iso_mesh();
    b->u = u;
    u->device = dev;
    DevMesh &d = u->dev;
    double *cxyz, *vol, *st_w, *palpha, *ccen;
    int32_t *cpt, *sface, *snbr, *lface, *cflags, *st_ptr, *st_cell, *dom_off;
    if (!dev_alloc(u, &cxyz, 24 * N) || !dev_alloc(u, &vol, N) || !dev_alloc(u, &st_w, S) || !dev_alloc(u, &ccen, 3 * N) ||
        !dev_alloc(u, &palpha, std::max<int64_t>(P, 1)) || !dev_alloc(u, &cpt, 8 * N) ||
        !dev_alloc(u, &sface, (int64_t)W * N) || !dev_alloc(u, &snbr, (int64_t)W * N) || !dev_alloc(u, &lface, 6 * N) ||
        !dev_alloc(u, &cflags, N) || !dev_alloc(u, &st_ptr, K + 1) || !dev_alloc(u, &st_cell, S) ||
        !dev_alloc(u, &dom_off, n + 1)) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble mesh allocation failed");
    }
    // members with cells other than hexahedra: every cell of the union takes its face loops from
    // cloop, a hexahedron's in the directions the hexahedron kernels take, so that each member still
    // computes bit for bit what it computes alone
    int32_t *cloop = nullptr;
    if (generic && !dev_alloc(u, &cloop, 6 * N)) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble mesh allocation failed");
    }
    std::vector<std::vector<int32_t>> hex_loops;  // host staging, alive until the copies are done
    // general polyhedra: their point, face and loop arrays concatenated, indices offset
    int32_t *cbig = nullptr, *bv_ptr = nullptr, *bv_cls = nullptr, *bf_ptr = nullptr, *bf_face = nullptr,
            *bf_planar = nullptr, *bl_ptr = nullptr, *bl_vtx = nullptr;
    double *bv_xyz = nullptr;
    if (any_big && (!dev_alloc(u, &cbig, N) || !dev_alloc(u, &bv_ptr, NB + 1) || !dev_alloc(u, &bv_cls, NBV) ||
                    !dev_alloc(u, &bv_xyz, 3 * NBV) || !dev_alloc(u, &bf_ptr, NB + 1) || !dev_alloc(u, &bf_face, NBF) ||
                    !dev_alloc(u, &bf_planar, NBF) || !dev_alloc(u, &bl_ptr, NBF + 1) || !dev_alloc(u, &bl_vtx, NBL))) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble mesh allocation failed");
    }
    // the update's 32-bit slot words, each member's as its own mesh has them, when some member has
    // them (they are relative to the member's cells, so they need no offsets: the member's first
    // cell and face offset go beside them); a member without them sends every slot to the full
    // tables
    bool words = false;
    for (int32_t i = 0; i < n; ++i) words = words || meshes[i]->dev.slot_nar != nullptr;
    int2 *spair = nullptr;
    if (!dev_alloc(u, &spair, (int64_t)W * N)) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble mesh allocation failed");
    }
    int32_t *snar = nullptr, *nar_dom = nullptr, *nar_blk = nullptr;
    const int64_t n_blk = (N + 63) / 64;
    if (words && (!dev_alloc(u, &snar, (int64_t)W * N) || !dev_alloc(u, &nar_dom, 3 * (int64_t)n) ||
                  !dev_alloc(u, &nar_blk, 8 * n_blk))) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble mesh allocation failed");
    }
    std::vector<int32_t> hnar_dom;
    int64_t bo = 0, vo = 0, bfo = 0, blo = 0;
    hipStream_t s = b->stream;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    int64_t co = 0, fo = 0, ko = 0, so = 0, po = 0;
    b->cell_off.push_back(0);
    b->face_off.push_back(0);
    for (int32_t i = 0; i < n; ++i) {
        const iso_mesh *m = meshes[i];
        const DevMesh &md = m->dev;
        const int64_t nc = m->n_cells;
        ok(hipMemcpyAsync(cxyz + 24 * co, md.cxyz, 24 * nc * sizeof(double), hipMemcpyDeviceToDevice, s));
        ok(hipMemcpyAsync(vol + co, md.vol, nc * sizeof(double), hipMemcpyDeviceToDevice, s));
        ok(hipMemcpyAsync(ccen + 3 * co, md.ccen, 3 * nc * sizeof(double), hipMemcpyDeviceToDevice, s));
        ok(hipMemcpyAsync(cflags + co, md.cflags, nc * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        ok(launch_offset_copy(md.cpt, cpt + 8 * co, 8 * nc, 0, (int32_t)ko, 0, s));
        for (int k = 0; k < W; ++k) {
            int32_t *df = sface + (size_t)k * N + co, *dn = snbr + (size_t)k * N + co;
            if (k < m->W) {
                ok(launch_offset_copy(md.slot_face + (size_t)k * nc, df, nc, 1, (int32_t)fo, 0, s));
                ok(launch_offset_copy(md.slot_nbr + (size_t)k * nc, dn, nc, 2, (int32_t)co, (int32_t)po, s));
            } else {
                ok(launch_offset_copy(nullptr, df, nc, 0, kEmpty, 0, s));
                ok(launch_offset_copy(nullptr, dn, nc, 0, -1, 0, s));
            }
        }
        if (words) {
            for (int k = 0; k < W; ++k) {
                int32_t *dw = snar + (size_t)k * N + co;
                if (k < m->W && md.slot_nar)
                    ok(hipMemcpyAsync(dw, md.slot_nar + (size_t)k * nc, nc * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
                else if (k < m->W)
                    ok(launch_offset_copy(nullptr, dw, nc, 0, 0xFFFF, 0, s));  // read from the full tables
                else
                    ok(launch_offset_copy(nullptr, dw, nc, 0, 0xFFFE, 0, s));  // empty slots
            }
            hnar_dom.push_back((int32_t)md.nar_S);
            hnar_dom.push_back((int32_t)fo);
            hnar_dom.push_back((int32_t)co);
        }
        ok(launch_offset_copy(md.lface, lface + 6 * co, 6 * nc, 1, (int32_t)fo, 0, s));
        if (cloop && md.cloop) {
            ok(hipMemcpyAsync(cloop + 6 * co, md.cloop, 6 * nc * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        } else if (cloop) {
            hex_loops.emplace_back(6 * (size_t)nc);
            std::vector<int32_t> &h = hex_loops.back();
            for (int64_t c = 0; c < nc; ++c)
                for (int k = 0; k < 6; ++k) h[6 * (size_t)c + k] = hex_loop_word(k);
            ok(hipMemcpyAsync(cloop + 6 * co, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        if (any_big && md.cbig) {
            ok(launch_offset_copy(md.cbig, cbig + co, nc, 0, (int32_t)bo, 0, s));
            ok(launch_offset_copy(md.bv_ptr, bv_ptr + bo, m->n_big, 0, (int32_t)vo, 0, s));
            ok(launch_offset_copy(md.bv_cls, bv_cls + vo, m->n_bv, 0, (int32_t)ko, 0, s));
            ok(hipMemcpyAsync(bv_xyz + 3 * vo, md.bv_xyz, 3 * (size_t)m->n_bv * sizeof(double), hipMemcpyDeviceToDevice, s));
            ok(launch_offset_copy(md.bf_ptr, bf_ptr + bo, m->n_big, 0, (int32_t)bfo, 0, s));
            ok(launch_offset_copy(md.bf_face, bf_face + bfo, m->n_bf, 1, (int32_t)fo, 0, s));
            ok(launch_offset_copy(md.bf_planar, bf_planar + bfo, m->n_bf, 0, 0, 0, s));
            ok(launch_offset_copy(md.bl_ptr, bl_ptr + bfo, m->n_bf, 0, (int32_t)blo, 0, s));
            ok(launch_offset_copy(md.bl_vtx, bl_vtx + blo, m->n_bl, 0, 0, 0, s));
            bo += m->n_big; vo += m->n_bv; bfo += m->n_bf; blo += m->n_bl;
        } else if (any_big) {
            ok(launch_offset_copy(nullptr, cbig + co, nc, 0, -1, 0, s));  // no polyhedron here
        }
        ok(launch_offset_copy(md.st_ptr, st_ptr + ko, m->n_classes, 0, (int32_t)so, 0, s));
        ok(launch_offset_copy(md.st_cell, st_cell + so, m->st_nnz, 0, (int32_t)co, 0, s));
        ok(hipMemcpyAsync(st_w + so, md.st_w, m->st_nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (md.n_patches > 0)
            ok(hipMemcpyAsync(palpha + po, md.patch_alpha, md.n_patches * sizeof(double), hipMemcpyDeviceToDevice, s));
        co += nc; fo += m->n_faces; ko += m->n_classes; so += m->st_nnz; po += md.n_patches;
        b->cell_off.push_back(co);
        b->face_off.push_back(fo);
    }
    std::vector<int32_t> hoff(b->cell_off.begin(), b->cell_off.end());
    const int32_t snnz = (int32_t)S;
    ok(hipStreamSynchronize(s));
    ok(hipMemcpy(st_ptr + K, &snnz, sizeof(int32_t), hipMemcpyHostToDevice));
    if (any_big) {  // the arrays' closing offsets
        const int32_t nbv = (int32_t)NBV, nbf = (int32_t)NBF, nbl = (int32_t)NBL;
        ok(hipMemcpy(bv_ptr + NB, &nbv, sizeof(int32_t), hipMemcpyHostToDevice));
        ok(hipMemcpy(bf_ptr + NB, &nbf, sizeof(int32_t), hipMemcpyHostToDevice));
        ok(hipMemcpy(bl_ptr + NBF, &nbl, sizeof(int32_t), hipMemcpyHostToDevice));
    }
    {  // the union's slots cell-major, from its slot tables (filled on the stream above)
        DevMesh t;
        t.n_cells = (int32_t)N;
        t.W = W;
        t.slot_face = sface;
        t.slot_nbr = snbr;
        ok(launch_slot_pairs(t, spair, s));
    }
    ok(hipMemcpy(dom_off, hoff.data(), hoff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (words) {
        // the record of each 64-cell block (the layout is described with DevMesh::nar_blk)
        std::vector<int32_t> hblk(8 * n_blk, 0);
        int32_t dm = 0;
        for (int64_t bk = 0; bk < n_blk; ++bk) {
            const int64_t c = 64 * bk, e = std::min<int64_t>(c + 64, N);
            while (dm + 1 < n && hoff[dm + 1] <= c) ++dm;
            int32_t split = 64;
            if (dm + 1 < n && hoff[dm + 1] < e) split = dm + 2 < n && hoff[dm + 2] < e ? -1 : (int32_t)(hoff[dm + 1] - c);
            int32_t *r = &hblk[8 * bk];
            for (int j = 0; j < 3; ++j) r[j] = hnar_dom[3 * dm + j];
            r[3] = split;
            if (dm + 1 < n)
                for (int j = 0; j < 3; ++j) r[4 + j] = hnar_dom[3 * (dm + 1) + j];
            r[7] = dm;
        }
        ok(hipMemcpy(nar_dom, hnar_dom.data(), hnar_dom.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        ok(hipMemcpy(nar_blk, hblk.data(), hblk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (e != hipSuccess) {
        iso_batch_destroy(b);
        return fail(ISO_EDEVICE, std::string("ensemble mesh assembly failed: ") + hipGetErrorString(e));
    }
    d.n_cells = (int32_t)N; d.n_faces = (int32_t)F; d.n_classes = (int32_t)K; d.W = W; d.n_patches = (int32_t)P;
    d.cxyz = cxyz; d.cpt = cpt; d.vol = vol; d.slot_face = sface; d.slot_nbr = snbr; d.lface = lface;
    d.slot_pair = spair;
    d.cflags = cflags; d.st_ptr = st_ptr; d.st_cell = st_cell; d.st_w = st_w; d.patch_alpha = palpha;
    d.ccen = ccen;
    d.cloop = cloop;
    d.n_dom = n; d.dom_off = dom_off;
    if (words) {
        d.slot_nar = reinterpret_cast<const uint32_t *>(snar);
        d.nar_dom = nar_dom;
        d.nar_blk = nar_blk;
    }
    u->generic = generic;
    if (any_big) {
        d.cbig = cbig; d.bv_ptr = bv_ptr; d.bv_cls = bv_cls; d.bv_xyz = bv_xyz; d.bf_ptr = bf_ptr;
        d.bf_face = bf_face; d.bf_planar = bf_planar; d.bl_ptr = bl_ptr; d.bl_vtx = bl_vtx;
        d.big_face_pts = big_face_pts;
        d.all_big = all_big ? 1 : 0;
        d.big_class = narrow && wide ? 2 : -1;
        u->n_big = (int32_t)NB; u->n_bv = (int32_t)NBV; u->n_bf = (int32_t)NBF; u->n_bl = (int32_t)NBL;
    }
    u->n_cells = (int32_t)N; u->n_faces = (int32_t)F; u->n_classes = (int32_t)K; u->W = W;
    u->n_flux = (int32_t)NF; u->st_nnz = S;

    iso_status st = iso_plan_create(u, opt, b->stream, &b->plan);
    if (st != ISO_OK) {
        b->plan = nullptr;
        iso_batch_destroy(b);
        return st;
    }
    b->cfg = launch_cfg(b->plan->opt);
    if (!dev_alloc(u, &b->dt_dev, n) || !dev_alloc(u, &b->tmp, N) ||
        hipHostMalloc((void **)&b->dt_host, sizeof(double) * n) != hipSuccess) {
        iso_batch_destroy(b);
        return fail(ISO_ENOMEM, "ensemble workspace allocation failed");
    }
    *out = b;
    return ISO_OK;
}

iso_status iso_batch_layout(const iso_batch *b, int64_t *cell_off, int64_t *face_off) {
    if (!b || !cell_off || !face_off) return fail(ISO_EINVAL, "null argument");
    std::memcpy(cell_off, b->cell_off.data(), sizeof(int64_t) * (b->n + 1));
    std::memcpy(face_off, b->face_off.data(), sizeof(int64_t) * (b->n + 1));
    return ISO_OK;
}

iso_status iso_batch_advect(iso_batch *b, double *alpha, const double *phi, int64_t phi_stride, const double *U,
                            int64_t U_stride, const double *dt, int32_t n_steps) {
    if (!b) return fail(ISO_EINVAL, "null ensemble");
    if (!alpha || !phi || !U || !dt) return fail(ISO_EINVAL, "null array");
    if (n_steps < 0) return fail(ISO_EINVAL, "negative step count");
    const int64_t N = b->u->n_cells, F = b->u->n_faces;
    if ((phi_stride != 0 && phi_stride < F) || (U_stride != 0 && U_stride < 3 * N) || phi_stride < 0 || U_stride < 0)
        return fail(ISO_EINVAL, "field strides must be 0 or at least one step's fields");
    if (n_steps == 0) return ISO_OK;
    const auto lo = reinterpret_cast<uintptr_t>(alpha), hi = lo + (uintptr_t)N * 8;
    auto hits = [&](const void *p, int64_t elems) {
        const auto x = reinterpret_cast<uintptr_t>(p);
        return x < hi && lo < x + (uintptr_t)elems * 8;
    };
    if (hits(phi, (n_steps - 1) * phi_stride + F) || hits(U, (n_steps - 1) * U_stride + 3 * N))
        return fail(ISO_EINVAL, "alpha overlaps the fields");
    // order after the caller's work on its stream
    if (hipEventRecord(b->ev_in, b->user) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
        return fail(ISO_EDEVICE, "stream ordering failed");
    iso_status st = upload_dt(b, dt);
    if (st != ISO_OK) return st;
    (void)hipGetLastError();
    hipError_t e = hipSuccess;
    if (n_steps > kMaxGraphSteps) {
        e = enqueue_steps(b, alpha, phi, phi_stride, U, U_stride, n_steps, b->cfg);
    } else {
        iso_batch::Key k;
        k.alpha = alpha; k.phi = phi; k.U = U; k.ps = phi_stride; k.us = U_stride; k.steps = n_steps; k.cfg = b->cfg;
        const bool hit = b->have_graph && k.alpha == b->key.alpha && k.phi == b->key.phi && k.U == b->key.U &&
                         k.ps == b->key.ps && k.us == b->key.us && k.steps == b->key.steps && same_cfg(k.cfg, b->key.cfg);
        if (!hit) {
            drop_graph(b);
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                hipError_t el = enqueue_steps(b, alpha, phi, phi_stride, U, U_stride, n_steps, b->cfg);
                e = hipStreamEndCapture(b->stream, &b->graph);
                if (el != hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return fail(ISO_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
            }
            b->key = k;
            b->have_graph = true;
        }
        e = hipGraphLaunch(b->exec, b->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->ev_out, 0);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("ensemble step failed: ") + hipGetErrorString(e));
    return ISO_OK;
}

iso_status iso_batch_config(const iso_batch *b, int32_t *cfg) {
    if (!b || !cfg) return fail(ISO_EINVAL, "null argument");
    cfg[0] = b->cfg.block_cells; cfg[1] = b->cfg.surface_blocks; cfg[2] = b->cfg.surface_waves;
    cfg[3] = b->cfg.bound_blocks;
    return ISO_OK;
}

iso_status iso_batch_set_config(iso_batch *b, const int32_t *cfg) {
    if (!b || !cfg) return fail(ISO_EINVAL, "null argument");
    if (cfg[0] < 1 || cfg[0] > 1024 || cfg[1] < 0 || cfg[1] > 65535 || cfg[2] < 1 || cfg[2] > 4 || cfg[3] < 1 ||
        cfg[3] > 65535)
        return fail(ISO_EINVAL, "launch shape out of range");
    LaunchCfg c = b->cfg;  // the launch shapes only: the options' choices (slot words) stay
    c.block_cells = cfg[0];
    c.surface_blocks = cfg[1];
    c.surface_waves = cfg[2];
    c.bound_blocks = cfg[3];
    b->cfg = c;
    return ISO_OK;
}

iso_status iso_batch_tune(iso_batch *b, const double *alpha, const double *phi, const double *U, const double *dt,
                          int32_t n_trial, const char *cache_path, double *best_ms) {
    if (!b || !alpha || !phi || !U || !dt) return fail(ISO_EINVAL, "null argument");
    if (n_trial < 1) return fail(ISO_EINVAL, "n_trial must be positive");
    const std::string sig = signature(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string key;
            int32_t c[4];
            double ms = 0;
            if (ls >> key >> c[0] >> c[1] >> c[2] >> c[3] >> ms && key == sig) {
                if (iso_batch_set_config(b, c) == ISO_OK) {
                    if (best_ms) *best_ms = ms;
                    return ISO_OK;
                }
            }
        }
    }
    const int64_t N = b->u->n_cells;
    if (!b->scratch && !dev_alloc(b->u, &b->scratch, N)) return fail(ISO_ENOMEM, "tuning buffer allocation failed");
    if (hipEventRecord(b->ev_in, b->user) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
        return fail(ISO_EDEVICE, "stream ordering failed");
    iso_status st = upload_dt(b, dt);
    if (st != ISO_OK) return st;
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return fail(ISO_EDEVICE, "event creation failed");
    auto trial = [&](const LaunchCfg &c, double *ms) -> hipError_t {
        hipError_t e = launch_copy_f64(alpha, b->scratch, N, b->stream);
        if (e == hipSuccess) e = enqueue_steps(b, b->scratch, phi, 0, U, 0, 1, c);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
        if (e == hipSuccess) e = enqueue_steps(b, b->scratch, phi, 0, U, 0, n_trial, c);
        if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, t0, t1);
        *ms = f / n_trial;
        return e;
    };
    // coordinate search: interface-kernel shape first, then the per-cell block, then bounding
    LaunchCfg best = b->cfg;
    double best_t = 0;
    hipError_t e = trial(best, &best_t);
    const int waves[] = {1, 2, 3};
    const int sblocks[] = {512, 1024, 2048, 4096};
    const int cblocks[] = {128, 256, 512};
    const int bblocks[] = {256, 512, 1024};
    for (int sw : waves)
        for (int sb : sblocks) {
            if (e != hipSuccess) break;
            LaunchCfg c = best;
            c.surface_waves = sw;
            c.surface_blocks = sb;
            double t;
            e = trial(c, &t);
            if (e == hipSuccess && t < best_t) { best_t = t; best = c; }
        }
    for (int bc : cblocks) {
        if (e != hipSuccess) break;
        LaunchCfg c = best;
        c.block_cells = bc;
        double t;
        e = trial(c, &t);
        if (e == hipSuccess && t < best_t) { best_t = t; best = c; }
    }
    for (int bb : bblocks) {
        if (e != hipSuccess) break;
        LaunchCfg c = best;
        c.bound_blocks = bb;
        double t;
        e = trial(c, &t);
        if (e == hipSuccess && t < best_t) { best_t = t; best = c; }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("tuning trial failed: ") + hipGetErrorString(e));
    b->cfg = best;
    if (best_ms) *best_ms = best_t;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << sig << ' ' << best.block_cells << ' ' << best.surface_blocks << ' ' << best.surface_waves << ' '
             << best.bound_blocks << ' ' << best_t << '\n';
    }
    if (hipEventRecord(b->ev_out, b->stream) != hipSuccess || hipStreamWaitEvent(b->user, b->ev_out, 0) != hipSuccess)
        return fail(ISO_EDEVICE, "stream ordering failed");
    return ISO_OK;
}

}  // extern "C"
