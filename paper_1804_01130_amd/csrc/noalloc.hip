// The advection step for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): iso_advect_step_noalloc runs
// the same kernels as iso_advect_step, with the step's workspace (interface list, the dV of
// interface-upwind faces, bounding lists, marks, correction buffers and counters) carved out of
// one file-scope device array instead of a plan's allocations.
//
// Each device holds its own copy of the array, at its own address, until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on that device (the
// array's name in host code is a host-side stand-in, not a device address).  Every call on a
// device shares that device's array: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <array>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace isoadv {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DeviceScratch {
    unsigned char *ptr = nullptr;  // device address of this device's copy of scratch
    // layout of the last call that completed its launches; the kernels leave the regions that must
    // start at zero (counters, marks, correction buffers) zeroed at the end of every step, so a call
    // with the same layout need not clear them again
    int64_t key[2] = {-1, -1};
};
std::array<DeviceScratch, kMaxDevices> g_scratch;
std::mutex g_scratch_mu;

__global__ void k_zero_words(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

struct Layout {
    size_t counters, surf, dvs, olist, tlist, flist, cmark, fmark, delta, dvcur, end;
};

Layout layout_for(int64_t nc, int64_t nf) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    Layout L{};
    size_t o = 0;
    L.counters = o; o = up(o + kCntNum * sizeof(int32_t));
    L.cmark = o; o = up(o + 2 * nc * sizeof(int32_t));     // zero between steps
    L.fmark = o; o = up(o + nf * sizeof(int32_t));         // zero between steps
    L.delta = o; o = up(o + 3 * nf * sizeof(double));      // zero between steps
    L.surf = o; o = up(o + nc * sizeof(int32_t));
    L.dvs = o; o = up(o + nf * sizeof(double));
    L.olist = o; o = up(o + nc * sizeof(int32_t));
    L.tlist = o; o = up(o + 2 * nc * sizeof(int32_t));
    L.flist = o; o = up(o + 4 * nf * sizeof(int32_t));
    L.dvcur = o; o = up(o + nf * sizeof(double));
    L.end = o;
    return L;
}

}  // namespace
}  // namespace isoadv

using namespace isoadv;

extern "C" iso_status iso_advect_step_noalloc(const iso_mesh *mesh, const iso_options *opt, void *stream,
                                              const double *alpha, const double *phi, const double *U, double dt,
                                              double *alpha_new) {
    if (!mesh) return fail(ISO_EINVAL, "null mesh");
    iso_options o;
    if (opt) o = *opt; else iso_options_default(&o);
    if (const iso_status so = check_options(o, mesh); so != ISO_OK) return so;
    if (o.check_inputs) return fail(ISO_EINVAL, "check_inputs copies the inputs to the host: not on this entry point");
    if (const iso_status sa = check_step_args(mesh, alpha, phi, U, dt, alpha_new, nullptr, nullptr); sa != ISO_OK)
        return sa;
    const int64_t nc = mesh->n_cells, nf = mesh->n_faces;
    const Layout L = layout_for(nc, nf);
    if (L.end > kScratchBytes)
        return fail(ISO_ENOSPACE, "the mesh needs " + std::to_string(L.end) + " bytes of step workspace; this entry point holds " +
                                      std::to_string(kScratchBytes) + " (about 24 B per cell and 60 B per face)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(ISO_EDEVICE, "no current device");
    if (dev != mesh->device) return fail(ISO_EINVAL, "the mesh lives on another device than the current one");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    DeviceScratch &ds = g_scratch[dev];
    if (!ds.ptr) {  // once per device, with that device current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return fail(ISO_EDEVICE, "no address for the step workspace on this device");
        ds.ptr = static_cast<unsigned char *>(p);
    }
    unsigned char *base = ds.ptr;
    (void)hipGetLastError();
    if (ds.key[0] != nc || ds.key[1] != nf) {
        // a new layout: clear what must start at zero (a fill kernel rather than a memset node, so
        // that a captured graph replays it correctly)
        ds.key[0] = ds.key[1] = -1;
        const int64_t words = (int64_t)(L.surf - L.counters) / 4;
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 4096)), dim3(256), 0, s,
                           reinterpret_cast<uint32_t *>(base + L.counters), words);
    }
    DevWork w;
    w.counters = reinterpret_cast<int32_t *>(base + L.counters);
    w.surf = reinterpret_cast<int32_t *>(base + L.surf);
    w.dvs = reinterpret_cast<double *>(base + L.dvs);
    w.olist = reinterpret_cast<int32_t *>(base + L.olist);
    w.tlist = reinterpret_cast<int32_t *>(base + L.tlist);
    w.flist = reinterpret_cast<int32_t *>(base + L.flist);
    w.cmark = reinterpret_cast<int32_t *>(base + L.cmark);
    w.fmark = reinterpret_cast<int32_t *>(base + L.fmark);
    w.delta = reinterpret_cast<double *>(base + L.delta);
    w.dvcur = reinterpret_cast<double *>(base + L.dvcur);
    w.red = nullptr;  // no statistics on this entry point
    w.cap = (int32_t)nc;  // every cell fits in the interface list
    StepArgs args{alpha, phi, U, alpha_new, dt, nullptr, nullptr, nullptr};
    const hipError_t e = launch_step(mesh->dev, w, step_params(o), args, nullptr, launch_cfg(o), false, s, nullptr);
    if (e != hipSuccess) return fail(ISO_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    ds.key[0] = nc;
    ds.key[1] = nf;
    return ISO_OK;
}
