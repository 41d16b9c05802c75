// swe_api.hip -- the extern "C" interface of libswe.so (declared in swe.h):
// argument validation, ownership of the library's device scratch, the
// asynchronous step loop and error reporting.  No C++ exception crosses the
// interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "swe.h"
#include "swe_internal.hpp"

using swe::Ctl;
using swe::Params;

struct swe_handle {
    Params P{};
    int dtype = SWE_F64;
    int path = SWE_PATH_FUSED;
    int H = 0, gy = 0;
    bool more_waves = false;   // the fused step's occupancy variant (SWE_FUSED_WAVES)
    bool split = true;         // two waves per tile (SWE_FUSED_SPLIT=0: one)
    int spin_cap = swe::kSplitSpinCap;   // the split step's bound on its waits
    int Ht = 0, gyt = 0;       // tile rows and chunks of the one-wave tracing step (swe_grad)
    size_t elem = 8;
    hipStream_t stream = nullptr;
    int device = 0;
    void* eta = nullptr;       // caller's state (buffer A)
    void* qx = nullptr;
    void* qy = nullptr;
    const void* z = nullptr;
    const void* n = nullptr;   // caller's Manning field (for the adjoint's dJ/dn)
    void* buf = nullptr;       // library: state buffer B (3 fields) + m
    Ctl* ctl = nullptr;
    double* part = nullptr;    // 2 * nparts
    int nparts = 0;
    double* hydro = nullptr;   // device copy of (t, q)
    std::vector<double> hydro_host;   // host copy: hydro_len times, then discharges
    void* trace = nullptr;     // unfused scratch: 47 padded arrays + zp + mp
    unsigned* dry = nullptr;   // dry-tile skip flags (2 * nparts words), or NULL
    void* fpart = nullptr;     // fused path: tile and group records, group tickets
    // swe_grad's kept trajectory (U^n, U*, U^d of every step), kept for the
    // next call: freeing a large buffer that kernels have written costs tens
    // of milliseconds per 100 GB, and more when another such free is pending
    void* traj = nullptr;
    size_t traj_bytes = 0;
    long long step_host = 0;
    std::string err;
};

namespace {

thread_local std::string g_create_err = "no error";

const char* hip_text(hipError_t e) { return hipGetErrorString(e); }

int fail(swe_handle* h, int code, const std::string& msg) {
    if (h)
        h->err = msg;
    else
        g_create_err = msg;
    return code;
}

int hip_fail(swe_handle* h, hipError_t e, const char* what) {
    return fail(h, SWE_EDEVICE, std::string(what) + ": " + hip_text(e));
}

size_t field_bytes(const swe_handle* h) {
    return (size_t)h->P.ny * (size_t)h->P.pitch * h->elem;
}

void* bufB(const swe_handle* h, int k) {  // k = 0 eta, 1 qx, 2 qy, 3 m
    return (char*)h->buf + (size_t)k * field_bytes(h);
}

void* bufA(const swe_handle* h, int k) {
    return k == 0 ? h->eta : (k == 1 ? h->qx : h->qy);
}

size_t padded_elems(const swe_handle* h) {
    return (size_t)(h->P.nx + 2) * (size_t)(h->P.ny + 2);
}

template <typename T>
__global__ void k_copy_back(const Ctl* ctl, T* a0, T* a1, T* a2, const T* b0, const T* b1,
                            const T* b2, size_t n) {
    if (!(ctl->call_steps & 1)) return;
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; k < n; k += stride) {
        a0[k] = b0[k];
        a1[k] = b1[k];
        a2[k] = b2[k];
    }
}

// If the steps of the current call ended in buffer B, copy it back to the
// caller's arrays (decided on the device, so the host never waits).
template <typename T>
hipError_t copy_back(swe_handle* h) {
    // the last row ends at nx: a pitched caller view may own nothing beyond it
    const size_t n = (size_t)(h->P.ny - 1) * (size_t)h->P.pitch + (size_t)h->P.nx;
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_copy_back<T>, dim3((unsigned)blocks), dim3(256), 0, h->stream, h->ctl,
                       (T*)bufA(h, 0), (T*)bufA(h, 1), (T*)bufA(h, 2), (const T*)bufB(h, 0),
                       (const T*)bufB(h, 1), (const T*)bufB(h, 2), n);
    return hipGetLastError();
}

// Enqueue the k-th step of a call: sigma follows the global step index, and
// even k read the caller's arrays (A) and write the library's (B).
template <typename T>
hipError_t enqueue_step(swe_handle* h, int64_t k, double t_end, bool unfused, double* log_dt,
                        double* log_t) {
    const int sigma = ((h->step_host + k) & 1) ? -1 : 1;
    const int s = k & 1;  // 0: A -> B, 1: B -> A
    const T* src[3];
    T* dst[3];
    for (int v = 0; v < 3; ++v) {
        src[v] = (const T*)(s ? bufB(h, v) : bufA(h, v));
        dst[v] = (T*)(s ? bufA(h, v) : bufB(h, v));
    }
    if (unfused) {
        swe::UnfusedArgs<T> a;
        a.P = h->P;
        a.ctl = h->ctl;
        a.t_end = t_end;
        a.eta = src[0]; a.qx = src[1]; a.qy = src[2];
        a.z = (const T*)h->z;
        a.eta1 = dst[0]; a.qx1 = dst[1]; a.qy1 = dst[2];
        a.trace = (T*)h->trace;
        a.zp = (const T*)h->trace + (size_t)swe::kTraceArrays * padded_elems(h);
        a.mp = a.zp + padded_elems(h);
        a.part_def = h->part;
        a.part_vol = h->part + h->nparts;
        return swe::launch_unfused_step<T>(a, sigma, h->stream);
    }
    swe::FusedArgs<T> a;
    a.P = h->P;
    a.ctl = h->ctl;
    a.t_end = t_end;
    a.eta = src[0]; a.qx = src[1]; a.qy = src[2];
    a.z = (const T*)h->z;
    a.m = (const T*)bufB(h, 3);
    a.eta1 = dst[0]; a.qx1 = dst[1]; a.qy1 = dst[2];
    swe::fused_part_layout(a, h->fpart, h->nparts);
    a.gy = h->gy;
    a.H = h->H;
    a.dry = h->dry;
    a.log_dt = log_dt;
    a.log_t = log_t;
    a.spin_cap = h->spin_cap;
    return swe::launch_fused<T>(a, sigma, h->stream, h->more_waves, h->split);
}

// Start of a host call: per-call statistics reset and, with the dry-tile
// skip on, every tile flag cleared (the caller may have changed the state
// since the last call, so the first step of a call computes every tile).
hipError_t begin_call(swe_handle* h, hipStream_t s) {
    return swe::launch_begin_call(h->ctl, s, h->dry, 2 * h->nparts);
}

// log_dt, log_t (fused path): where the step stores its dt^n and t^n, or NULL.
hipError_t enqueue(swe_handle* h, int64_t k, double t_end, bool unfused,
                   double* log_dt = nullptr, double* log_t = nullptr) {
    return h->dtype == SWE_F32 ? enqueue_step<float>(h, k, t_end, unfused, log_dt, log_t)
                               : enqueue_step<double>(h, k, t_end, unfused, log_dt, log_t);
}

hipError_t enqueue_copy_back(swe_handle* h) {
    return h->dtype == SWE_F32 ? copy_back<float>(h) : copy_back<double>(h);
}

int ensure_trace(swe_handle* h) {
    if (h->trace) return SWE_OK;
    const size_t bytes = (size_t)(swe::kTraceArrays + 2) * padded_elems(h) * h->elem;
    hipError_t e = hipMalloc(&h->trace, bytes);
    if (e != hipSuccess) {
        h->trace = nullptr;
        return fail(h, SWE_ENOMEM, std::string("hipMalloc of the unfused scratch failed: ") +
                                       hip_text(e));
    }
    e = hipMemsetAsync(h->trace, 0, bytes, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemsetAsync");
    void* zp = (char*)h->trace + (size_t)swe::kTraceArrays * padded_elems(h) * h->elem;
    void* mp = (char*)zp + padded_elems(h) * h->elem;
    e = h->dtype == SWE_F32
            ? swe::launch_pad_static<float>(h->P, (const float*)h->z, (const float*)bufB(h, 3),
                                            (float*)zp, (float*)mp, h->stream)
            : swe::launch_pad_static<double>(h->P, (const double*)h->z,
                                             (const double*)bufB(h, 3), (double*)zp, (double*)mp,
                                             h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "padding the static fields");
    return SWE_OK;
}

int fill_stats(swe_handle* h, swe_stats* out) {
    Ctl c;
    hipError_t e = hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reading the control block");
    h->step_host = c.step;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->step = c.step;
        out->steps = c.call_steps;
        out->bad_step = c.bad_step;
        out->flags = c.flags;
        out->t = c.t;
        out->dt = c.dt;
        out->dt_min = c.call_steps > 0 ? c.dt_min : 0.0;
        out->dt_max = c.dt_max_used;
        out->volume = c.volume;
        out->defect = c.defect;
        out->lambda_max = c.lam_max;
        out->cells_skipped = (int64_t)c.skipped;
    }
    if (c.flags & swe::FLAG_FATAL) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "unstable: flags 0x%x raised at step %lld", c.flags,
                      (long long)c.bad_step);
        return fail(h, SWE_EUNSTABLE, buf);
    }
    return SWE_OK;
}

bool is_device_ptr(const void* p, int device) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == device;
}

// Rows per fused workgroup: as many chunks per strip as there are resident
// wave slots on the device, so the whole grid runs in one round of waves (a
// partial second round would leave most of the GPU idle), but never fewer
// than 6 rows.  A wave's time is about proportional to the H + 4 rows it
// marches (the two-row halo at each chunk end included), so on grids too
// small to fill the slots the shortest chunks win (measured on MI355X: 1024^2
// FP64 36 us per step at 10 rows against 46 us at 16; 256^2 19 us at 6 rows
// against 34 us at 16).  With the dry-tile skip at most 32 rows: smaller
// tiles follow the wet/dry front more closely, and the skipped ones free
// their wave slot at once.
int auto_tile_rows(const swe_handle* h, int dev, bool dry_skip, bool one_wave = false) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    const int per_cu =
        h->split && !h->more_waves && !one_wave
            ? (h->dtype == SWE_F32 ? swe::fused_split_tiles_per_cu<float>()
                                   : swe::fused_split_tiles_per_cu<double>())
            : (h->dtype == SWE_F32 ? swe::fused_waves_per_cu<float>(h->more_waves)
                                   : swe::fused_waves_per_cu<double>(h->more_waves));
    return swe::fused_auto_rows(h->P.nx, h->P.ny, (long long)cus * per_cu, dry_skip);
}

int validate(const swe_config* c, std::string& why) {
    auto bad = [&](const char* m) {
        why = m;
        return SWE_EINVAL;
    };
    if (!c) return bad("config is NULL");
    if (c->nx < 5 || c->ny < 5) return bad("nx and ny must be >= 5");
    if ((long long)c->nx * (long long)c->ny > (1ll << 31)) return bad("grid larger than 2^31 cells");
    if (c->dtype != SWE_F32 && c->dtype != SWE_F64) return bad("dtype must be SWE_F32 or SWE_F64");
    if (c->path != SWE_PATH_FUSED && c->path != SWE_PATH_UNFUSED) return bad("unknown path");
    if (c->pitch < c->nx) return bad("pitch must be >= nx");
    if (!(c->dx > 0) || !(c->dy > 0) || !std::isfinite(c->dx) || !std::isfinite(c->dy))
        return bad("dx and dy must be finite and > 0");
    if (!(c->g > 0) || !std::isfinite(c->g)) return bad("g must be finite and > 0");
    if (!(c->cfl > 0) || !(c->cfl <= 1)) return bad("cfl must be in (0, 1]");
    if (!(c->h_dry >= 0) || !std::isfinite(c->h_dry)) return bad("h_dry must be >= 0");
    if (!(c->kappa >= 0) || !(c->kappa <= 4)) return bad("kappa must be in [0, 4]");
    if (!(c->eps_max >= 0) || !(c->eps_max <= 0.25)) return bad("eps_max must be in [0, 0.25]");
    if (!(c->dt_max > 0) || !std::isfinite(c->dt_max)) return bad("dt_max must be finite and > 0");
    if (std::isnan(c->dt_fixed) || std::isinf(c->dt_fixed)) return bad("dt_fixed must be finite");
    if (!std::isfinite(c->t0)) return bad("t0 must be finite");
    if (c->tile_rows < 0 || c->tile_rows > 65536) return bad("tile_rows out of range");
    if (c->dry_skip != 0 && c->dry_skip != 1) return bad("dry_skip must be 0 or 1");
    if (c->dry_skip && c->path != SWE_PATH_FUSED) return bad("dry_skip needs the fused path");
    if (!(c->h_film >= 0.0) || !std::isfinite(c->h_film)) return bad("h_film must be finite and >= 0");
    for (int k = 0; k < 4; ++k) {
        if (c->bc[k] < SWE_BC_WALL || c->bc[k] > SWE_BC_INFLOW) return bad("unknown boundary kind");
    }
    if (c->hydro_len < 0 || c->hydro_len > swe::kMaxHydro) return bad("hydro_len out of range");
    if (c->hydro_len > 0) {
        if (!c->hydro_t || !c->hydro_q) return bad("hydrograph pointers are NULL");
        for (int k = 0; k < c->hydro_len; ++k) {
            if (!std::isfinite(c->hydro_t[k]) || !std::isfinite(c->hydro_q[k]))
                return bad("hydrograph values must be finite");
            if (k > 0 && !(c->hydro_t[k] > c->hydro_t[k - 1]))
                return bad("hydrograph times must increase");
        }
    }
    if (!c->z || !c->n || !c->eta || !c->qx || !c->qy) return bad("a field pointer is NULL");
    return SWE_OK;
}

// A device is present and every field is device memory of the current one.
int check_device(const swe_config* c, int* dev, std::string& why) {
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        why = "no HIP device is available";
        return SWE_EDEVICE;
    }
    if ((e = hipGetDevice(dev)) != hipSuccess) {
        why = std::string("hipGetDevice: ") + hip_text(e);
        return SWE_EDEVICE;
    }
    const void* ptrs[5] = {c->z, c->n, c->eta, c->qx, c->qy};
    for (const void* p : ptrs)
        if (!is_device_ptr(p, *dev)) {
            why = "a field pointer is not device memory of the current device";
            return SWE_EDEVICE;
        }
    return SWE_OK;
}

// Host-side part of a handle: the caller's pointers, the parameter block,
// the tile layout and the host copy of the hydrograph (no device memory).
void prepare_handle(swe_handle* h, const swe_config* c, int dev) {
    h->dtype = c->dtype;
    h->elem = c->dtype == SWE_F32 ? 4 : 8;
    h->path = c->path;
    h->stream = (hipStream_t)c->stream;
    h->device = dev;
    h->eta = c->eta;
    h->qx = c->qx;
    h->qy = c->qy;
    h->z = c->z;
    h->n = c->n;
    Params& P = h->P;
    P.nx = c->nx;
    P.ny = c->ny;
    P.pitch = c->pitch;
    for (int k = 0; k < 4; ++k) {
        P.bc[k] = c->bc[k];
        P.lo[k] = c->inflow_lo[k];
        P.hi[k] = c->inflow_hi[k];
    }
    P.hydro_len = c->hydro_len;
    P.dx = c->dx; P.dy = c->dy; P.g = c->g; P.cfl = c->cfl; P.h_dry = c->h_dry;
    P.kappa = c->kappa; P.eps_max = c->eps_max; P.dt_max = c->dt_max; P.dt_fixed = c->dt_fixed;
    P.idx = 1.0 / c->dx;
    P.idy = 1.0 / c->dy;
    P.rcap = c->h_film > 0.0 ? 1.0 / c->h_film : INFINITY;
    // SWE_FUSED_WAVES=3 (FP64) or 5 (FP32) in the environment selects the fused
    // step's occupancy variant, one resident wave per SIMD more than its
    // default register budget allows (a measurement knob; same results)
    if (const char* w = std::getenv("SWE_FUSED_WAVES"))
        h->more_waves = c->path == SWE_PATH_FUSED && c->dry_skip == 0 &&
                        std::atoi(w) == (c->dtype == SWE_F32 ? 5 : 3);
    // SWE_FUSED_SPLIT=0 in the environment runs the fused step with one wave
    // per tile instead of two (a measurement knob; same state bits)
    if (const char* sp = std::getenv("SWE_FUSED_SPLIT")) h->split = std::atoi(sp) != 0;
    // SWE_SPLIT_SPIN_CAP lowers the split step's bound on its waits (tests of
    // the stall report)
    if (const char* cap = std::getenv("SWE_SPLIT_SPIN_CAP"))
        h->spin_cap = std::max(0, std::min(swe::kSplitSpinCap, std::atoi(cap)));
    h->H = c->tile_rows > 0 ? c->tile_rows : auto_tile_rows(h, dev, c->dry_skip != 0);
    h->gy = (c->ny + h->H - 1) / h->H;
    // swe_grad's tracing step runs one wave per tile, at that form's own
    // automatic height
    h->Ht = c->tile_rows > 0 ? c->tile_rows : auto_tile_rows(h, dev, false, true);
    // SWE_TRACE_ROWS fixes that height (a measurement knob; same bits)
    if (const char* tr = std::getenv("SWE_TRACE_ROWS"))
        if (std::atoi(tr) > 0) h->Ht = std::atoi(tr);
    h->gyt = (c->ny + h->Ht - 1) / h->Ht;
    h->nparts = std::max({swe::fused_blocks(c->nx, c->ny, h->H), swe::fused_blocks(c->nx, c->ny, h->Ht),
                          swe::scan_partials(c->nx, c->ny)});
    std::vector<double> hy(2 * (size_t)std::max(1, c->hydro_len), 0.0);
    for (int k = 0; k < c->hydro_len; ++k) {
        hy[k] = c->hydro_t[k];
        hy[c->hydro_len + k] = c->hydro_q[k];
    }
    h->hydro_host = hy;
}

// Device-side start of a handle whose scratch pointers are set: the
// hydrograph, m = g n^2, the control block at t0 and dt^0 from the state.
hipError_t init_device_state(swe_handle* h, const swe_config* c) {
    Params& P = h->P;
    hipError_t e = hipMemcpyAsync(h->hydro, h->hydro_host.data(),
                                  h->hydro_host.size() * sizeof(double), hipMemcpyHostToDevice,
                                  h->stream);
    P.hydro_t = h->hydro;
    P.hydro_q = h->hydro + std::max(0, c->hydro_len);
    if (e == hipSuccess)
        e = h->dtype == SWE_F32
                ? swe::launch_manning_m<float>(P, (const float*)c->n, (float*)bufB(h, 3), h->stream)
                : swe::launch_manning_m<double>(P, (const double*)c->n, (double*)bufB(h, 3),
                                                h->stream);
    if (e == hipSuccess) e = swe::launch_init_ctl(h->ctl, c->t0, 0, 0u, 0.0, h->stream);
    if (e == hipSuccess)
        e = h->dtype == SWE_F32
                ? swe::launch_scan<float>(P, h->ctl, INFINITY, (const float*)c->eta,
                                          (const float*)c->qx, (const float*)c->qy,
                                          (const float*)c->z, h->part, h->part + h->nparts, 0,
                                          h->stream)
                : swe::launch_scan<double>(P, h->ctl, INFINITY, (const double*)c->eta,
                                           (const double*)c->qx, (const double*)c->qy,
                                           (const double*)c->z, h->part, h->part + h->nparts, 0,
                                           h->stream);
    return e;
}

// ---------------------------------------------------- allocation-free run
//
// swe_run_noalloc keeps all of its device scratch (the second state buffer
// and m = g n^2, the control block, the partial sums and tickets, the
// hydrograph) in the file-scope array below instead of allocating it.
// Its largest grid has pitch * ny <= kNoAllocMaxElems and at most
// kNoAllocMaxTiles tiles.  The array exists once per device that loads this
// library and lives until the process ends.  Host code never passes its name
// to a kernel: the name is a host-side stand-in, and the device address comes
// from hipGetSymbolAddress, once per device (noalloc_scratch).
constexpr size_t kNoAllocMaxElems = size_t(1) << 20;
constexpr int kNoAllocMaxTiles = 1 << 16;
constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNoAllocStateBytes = al256(4 * kNoAllocMaxElems * sizeof(double));
constexpr size_t kNoAllocCtlBytes = al256(sizeof(Ctl));
constexpr size_t kNoAllocPartBytes = al256(2 * sizeof(double) * kNoAllocMaxTiles);
constexpr size_t kNoAllocGroups = (kNoAllocMaxTiles + swe::kGroup - 1) / swe::kGroup;
constexpr size_t kNoAllocFpartBytes =
    al256((kNoAllocMaxTiles + kNoAllocGroups) * sizeof(swe::TilePart) + kNoAllocGroups * sizeof(unsigned));
constexpr size_t kNoAllocHydroBytes = al256(2 * sizeof(double) * swe::kMaxHydro);
constexpr size_t kNoAllocBytes = kNoAllocStateBytes + kNoAllocCtlBytes + kNoAllocPartBytes +
                                 kNoAllocFpartBytes + kNoAllocHydroBytes;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

__global__ void k_zero16(uint4* p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        p[k] = make_uint4(0u, 0u, 0u, 0u);
}

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of `scratch` per device

// Device address of this device's copy of `scratch` (the current device).
int noalloc_scratch(int dev, void** out, std::string& why) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0) {
        why = "bad device index";
        return SWE_EDEVICE;
    }
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            why = std::string("hipGetSymbolAddress of the static scratch: ") + hip_text(e);
            return SWE_EDEVICE;
        }
        g_scratch_ptr[(size_t)dev] = p;
    }
    *out = g_scratch_ptr[(size_t)dev];
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_abi_version(void) { return SWE_ABI_VERSION; }

void swe_config_init(swe_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->dtype = SWE_F64;
    c->path = SWE_PATH_FUSED;
    c->g = 9.81;
    c->cfl = 0.5;
    c->h_dry = 1e-3;
    c->kappa = 0.5;
    c->eps_max = 0.25;
    c->dt_max = 1.0;
    c->dt_fixed = 0.0;
    c->t0 = 0.0;
    for (int k = 0; k < 4; ++k) {
        c->bc[k] = SWE_BC_WALL;
        c->inflow_lo[k] = 0;
        c->inflow_hi[k] = INT32_MAX;
    }
}

int swe_create(const swe_config* c, swe_handle** out) {
    if (!out) return fail(nullptr, SWE_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    int rc = validate(c, why);
    if (rc) return fail(nullptr, rc, why);
    int dev = 0;
    if ((rc = check_device(c, &dev, why)) != SWE_OK) return fail(nullptr, rc, why);

    swe_handle* h = new (std::nothrow) swe_handle();
    if (!h) return fail(nullptr, SWE_ENOMEM, "host allocation failed");
    prepare_handle(h, c, dev);

    auto cleanup = [&](int code) {
        swe_destroy(h);
        return code;
    };
    hipError_t e;
    if ((e = hipMalloc(&h->buf, 4 * field_bytes(h))) != hipSuccess) {
        h->buf = nullptr;
        fail(nullptr, SWE_ENOMEM, std::string("hipMalloc of the state buffer failed: ") + hip_text(e));
        return cleanup(SWE_ENOMEM);
    }
    if ((e = hipMalloc((void**)&h->ctl, sizeof(Ctl))) != hipSuccess ||
        (e = hipMalloc((void**)&h->part, 2 * sizeof(double) * (size_t)h->nparts)) != hipSuccess) {
        fail(nullptr, SWE_ENOMEM, std::string("hipMalloc failed: ") + hip_text(e));
        return cleanup(SWE_ENOMEM);
    }
    if ((e = hipMalloc((void**)&h->hydro, h->hydro_host.size() * sizeof(double))) != hipSuccess) {
        fail(nullptr, SWE_ENOMEM, std::string("hipMalloc failed: ") + hip_text(e));
        return cleanup(SWE_ENOMEM);
    }
    if (c->dry_skip) {
        if ((e = hipMalloc((void**)&h->dry, 2 * sizeof(unsigned) * (size_t)h->nparts)) != hipSuccess) {
            h->dry = nullptr;
            fail(nullptr, SWE_ENOMEM, std::string("hipMalloc failed: ") + hip_text(e));
            return cleanup(SWE_ENOMEM);
        }
    }
    if ((e = hipMalloc(&h->fpart, swe::fused_part_bytes(h->nparts))) != hipSuccess) {
        h->fpart = nullptr;
        fail(nullptr, SWE_ENOMEM, std::string("hipMalloc failed: ") + hip_text(e));
        return cleanup(SWE_ENOMEM);
    }
    e = hipMemsetAsync(h->fpart, 0, swe::fused_part_bytes(h->nparts), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->part, 0, 2 * sizeof(double) * h->nparts, h->stream);
    if (e == hipSuccess) e = init_device_state(h, c);
    if (e == hipSuccess && h->path == SWE_PATH_UNFUSED) {
        int rc2 = ensure_trace(h);
        if (rc2) {
            fail(nullptr, rc2, h->err);
            return cleanup(rc2);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        hip_fail(nullptr, e, "swe_create");
        return cleanup(SWE_EDEVICE);
    }
    h->step_host = 0;
    *out = h;
    return SWE_OK;
}

void swe_destroy(swe_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->buf) (void)hipFree(h->buf);
    if (h->ctl) (void)hipFree(h->ctl);
    if (h->part) (void)hipFree(h->part);
    if (h->hydro) (void)hipFree(h->hydro);
    if (h->trace) (void)hipFree(h->trace);
    if (h->dry) (void)hipFree(h->dry);
    if (h->fpart) (void)hipFree(h->fpart);
    if (h->traj) (void)hipFree(h->traj);
    delete h;
}

int swe_run(swe_handle* h, int64_t nsteps, double t_end, swe_stats* out) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(h, SWE_EINVAL, "nsteps must be >= 0");
    if (std::isnan(t_end)) return fail(h, SWE_EINVAL, "t_end is NaN");
    const bool unfused = h->path == SWE_PATH_UNFUSED;
    hipError_t e = begin_call(h, h->stream);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) e = enqueue(h, k, t_end, unfused);
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e != hipSuccess) return hip_fail(h, e, "launching the step kernels");
    return fill_stats(h, out);
}

int swe_run_noalloc(const swe_config* c, int64_t nsteps, double t_end, swe_stats* out) {
    std::string why;
    int rc = validate(c, why);
    if (rc) return fail(nullptr, rc, why);
    if (c->path != SWE_PATH_FUSED) return fail(nullptr, SWE_EINVAL, "swe_run_noalloc runs the fused path only");
    if (c->dry_skip) return fail(nullptr, SWE_EINVAL, "swe_run_noalloc does not take the dry-tile skip");
    if (nsteps < 0) return fail(nullptr, SWE_EINVAL, "nsteps must be >= 0");
    if (std::isnan(t_end)) return fail(nullptr, SWE_EINVAL, "t_end is NaN");
    if ((size_t)c->pitch * (size_t)c->ny > kNoAllocMaxElems)
        return fail(nullptr, SWE_EINVAL,
                    "grid too large for swe_run_noalloc: pitch * ny must be <= 1048576");
    int dev = 0;
    if ((rc = check_device(c, &dev, why)) != SWE_OK) return fail(nullptr, rc, why);
    void* base = nullptr;
    if ((rc = noalloc_scratch(dev, &base, why)) != SWE_OK) return fail(nullptr, rc, why);

    swe_handle h;   // host-side only: its device pointers all point into `scratch`
    prepare_handle(&h, c, dev);
    if (h.nparts > kNoAllocMaxTiles)
        return fail(nullptr, SWE_EINVAL, "too many tiles for swe_run_noalloc (tile_rows too small)");
    char* p = (char*)base;
    h.buf = p;
    p += kNoAllocStateBytes;
    h.ctl = (Ctl*)p;
    p += kNoAllocCtlBytes;
    h.part = (double*)p;
    p += kNoAllocPartBytes;
    h.fpart = p;
    p += kNoAllocFpartBytes;
    h.hydro = (double*)p;
    // every call shares the array: the tickets and partial sums of the last
    // call are cleared (a fill kernel, no memset node)
    const size_t nz16 = (kNoAllocPartBytes + kNoAllocFpartBytes) / 16;
    hipLaunchKernelGGL(k_zero16, dim3(256), dim3(256), 0, h.stream, (uint4*)h.part, nz16);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = init_device_state(&h, c);
    if (e == hipSuccess) e = begin_call(&h, h.stream);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) e = enqueue(&h, k, t_end, false);
    if (e == hipSuccess) e = enqueue_copy_back(&h);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(h.stream);
        return fail(nullptr, SWE_EDEVICE, std::string("swe_run_noalloc: ") + hip_text(e));
    }
    rc = fill_stats(&h, out);   // synchronises (the hydrograph copy reads h's host vector)
    if (rc != SWE_OK) fail(nullptr, rc, h.err);
    return rc;
}

int swe_run_dt(swe_handle* h, int64_t nsteps, const double* dts, swe_stats* out) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(h, SWE_EINVAL, "nsteps must be >= 0");
    if (nsteps > 0 && !dts) return fail(h, SWE_EINVAL, "dts is NULL");
    for (int64_t k = 0; k < nsteps; ++k)
        if (!(dts[k] > 0.0) || !std::isfinite(dts[k]))
            return fail(h, SWE_EINVAL, "every prescribed time step must be finite and > 0");
    const bool unfused = h->path == SWE_PATH_UNFUSED;
    hipError_t e = begin_call(h, h->stream);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        e = swe::launch_set_dt(h->P, h->ctl, dts[k], h->stream);
        if (e == hipSuccess) e = enqueue(h, k, INFINITY, unfused);
    }
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e != hipSuccess) return hip_fail(h, e, "launching the step kernels");
    return fill_stats(h, out);
}

int swe_step(swe_handle* h, double* dt_used) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    double dt_before = 0.0;
    if (dt_used) {
        Ctl c;
        hipError_t e = hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "reading the control block");
        dt_before = c.dt;
    }
    hipError_t e = begin_call(h, h->stream);
    if (e == hipSuccess) e = enqueue(h, 0, INFINITY, h->path == SWE_PATH_UNFUSED);
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e != hipSuccess) return hip_fail(h, e, "launching the step kernels");
    h->step_host += 1;
    if (dt_used) {
        int rc = fill_stats(h, nullptr);
        *dt_used = dt_before;
        return rc;
    }
    return SWE_OK;
}

int swe_get_stats(swe_handle* h, swe_stats* out) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (!out) return fail(h, SWE_EINVAL, "out is NULL");
    return fill_stats(h, out);
}

size_t swe_trace_bytes(const swe_handle* h) {
    if (!h) return 0;
    return (size_t)swe::kTraceArrays * padded_elems(h) * h->elem;
}

int swe_trace_step(swe_handle* h, void* arrays, size_t bytes, double* scalars) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (!arrays || !scalars) return fail(h, SWE_EINVAL, "arrays or scalars is NULL");
    if (bytes < swe_trace_bytes(h)) return fail(h, SWE_EINVAL, "trace buffer too small");
    if (!is_device_ptr(arrays, h->device)) return fail(h, SWE_EINVAL, "arrays is not device memory");
    int rc = ensure_trace(h);
    if (rc) return rc;
    Ctl before, after;
    hipError_t e = hipMemcpyAsync(&before, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = begin_call(h, h->stream);
    if (e == hipSuccess) e = enqueue(h, 0, INFINITY, true);
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e == hipSuccess)
        e = hipMemcpyAsync(arrays, h->trace, swe_trace_bytes(h), hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&after, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_trace_step");
    h->step_host = after.step;
    for (int k = 0; k < 16; ++k) scalars[k] = 0.0;
    scalars[0] = before.qin0;
    scalars[1] = before.qin1;
    scalars[2] = before.rx;
    scalars[3] = before.ry;
    scalars[4] = after.last_defect_depth;
    scalars[5] = after.lam_max;
    scalars[6] = after.dt;
    scalars[7] = after.volume;
    scalars[8] = (double)after.last_step_flags;
    scalars[9] = (before.step & 1) ? -1.0 : 1.0;
    scalars[10] = after.t;
    if (after.flags & swe::FLAG_FATAL) return fail(h, SWE_EUNSTABLE, "unstable step");
    return SWE_OK;
}

int swe_save(swe_handle* h, swe_checkpoint* ck) {
    if (!h || !ck) return fail(h, SWE_EINVAL, "handle or checkpoint is NULL");
    Ctl c;
    hipError_t e = hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_save");
    std::memset(ck, 0, sizeof(*ck));
    ck->step = c.step;
    ck->flags = c.flags;
    ck->t = c.t;
    ck->dt = c.dt;
    ck->defect = c.defect;
    return SWE_OK;
}

int swe_load(swe_handle* h, const swe_checkpoint* ck) {
    if (!h || !ck) return fail(h, SWE_EINVAL, "handle or checkpoint is NULL");
    if (!std::isfinite(ck->t) || ck->step < 0) return fail(h, SWE_EINVAL, "bad checkpoint");
    hipError_t e = swe::launch_init_ctl(h->ctl, ck->t, ck->step, ck->flags, ck->defect, h->stream);
    if (e == hipSuccess)
        e = h->dtype == SWE_F32
                ? swe::launch_scan<float>(h->P, h->ctl, INFINITY, (const float*)h->eta,
                                          (const float*)h->qx, (const float*)h->qy,
                                          (const float*)h->z, h->part, h->part + h->nparts, 0,
                                          h->stream)
                : swe::launch_scan<double>(h->P, h->ctl, INFINITY, (const double*)h->eta,
                                           (const double*)h->qx, (const double*)h->qy,
                                           (const double*)h->z, h->part, h->part + h->nparts, 0,
                                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_load");
    h->step_host = ck->step;
    return SWE_OK;
}

}  // extern "C"

namespace {

struct DevBuf {
    void* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
    double* d() const { return (double*)p; }
};

// Elements of a pitched field that belong to it (the last row ends at nx).
size_t state_elems(const swe_handle* h) {
    return (size_t)(h->P.ny - 1) * (size_t)h->P.pitch + (size_t)h->P.nx;
}

template <typename T>
hipError_t copy_state(swe_handle* h, T* const dst[3], const T* const src[3],
                      hipStream_t st = nullptr) {
    hipError_t e = hipSuccess;
    for (int f = 0; f < 3 && e == hipSuccess; ++f)
        e = hipMemcpyAsync(dst[f], src[f], state_elems(h) * sizeof(T), hipMemcpyDeviceToDevice,
                           st ? st : h->stream);
    return e;
}

// A second stream and the events between it and the handle's stream, for the
// reverse sweep's overlapped segment recompute; it drains its stream before
// the buffers it writes are freed.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t done[2] = {nullptr, nullptr};   // recompute into buffer b finished
    hipEvent_t freed[2] = {nullptr, nullptr};  // march out of buffer b finished
    bool used[2] = {false, false};
    hipError_t init() {
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        for (int b = 0; b < 2 && e == hipSuccess; ++b) {
            e = hipEventCreateWithFlags(&done[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&freed[b], hipEventDisableTiming);
        }
        return e;
    }
    SideStream() = default;
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
    ~SideStream() {
        if (s) (void)hipStreamSynchronize(s);
        for (int b = 0; b < 2; ++b) {
            if (done[b]) (void)hipEventDestroy(done[b]);
            if (freed[b]) (void)hipEventDestroy(freed[b]);
        }
        if (s) (void)hipStreamDestroy(s);
    }
};

// The discrete adjoint of nsteps steps of handle h, whose state has type T.
// The forward run, its checkpoints and the recomputed segments are in T; the
// reverse sweep is in FP64.  For T = float each step is linearised at its
// FP32 state promoted to FP64: the FP64 replay and adjoint of that step use
// the FP32 run's time step and FP64 copies of z, n and m = g n^2.
template <typename T>
int grad_impl(swe_handle* h, int64_t nsteps, const swe_gauges* g, int32_t ckpt_every,
              double* loss, void* dJ_dn, void* dJ_dz) {
    constexpr bool mixed = sizeof(T) == 4;
    // SWE_VERBOSE=1 in the environment: lines on stderr with the elapsed time
    // after the set-up, the forward run, each reverse segment and the end
    // (each waits for the device)
    const char* verbose_env = std::getenv("SWE_VERBOSE");
    const bool verbose = verbose_env && verbose_env[0] == '1';
    const auto t_start = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point t0) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    };
    const int64_t nobs = nsteps / g->obs_every;
    const int ng = g->ngauge;
    int rc = fill_stats(h, nullptr);
    if (rc) return rc;
    Ctl c0;
    hipError_t e = hipMemcpyAsync(&c0, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_grad: reading the control block");
    const long long step0 = c0.step;
    const size_t fe = (size_t)h->P.ny * (size_t)h->P.pitch;   // elements of a field slot
    const size_t Npad = padded_elems(h);
    // ckpt_every = 0: an FP64 handle keeps the whole trajectory (U^n, U* and
    // U^d of every step, 9 fields a step) when it fits in three quarters of
    // the free device memory: the forward run writes it, and the reverse
    // sweep recomputes nothing.  Otherwise, and for FP32 handles, checkpoints
    // every round(sqrt(nsteps)) steps.
    bool store_all = false;
    if (ckpt_every == 0 && !mixed && nsteps > 0) {
        const size_t need = (size_t)nsteps * 9 * fe * sizeof(double);
        if (h->traj_bytes >= need) {
            store_all = true;
        } else {
            size_t freeb = 0, totalb = 0;
            if (hipMemGetInfo(&freeb, &totalb) == hipSuccess &&
                (double)need <= 0.75 * (double)(freeb + h->traj_bytes)) {
                if (h->traj) (void)hipFree(h->traj);
                h->traj = nullptr;
                h->traj_bytes = 0;
                if (hipMalloc(&h->traj, need) == hipSuccess) {
                    h->traj_bytes = need;
                    store_all = true;
                } else {
                    h->traj = nullptr;
                }
            }
            (void)hipGetLastError();
        }
    }
    double* const traj_base = (double*)h->traj;
    const int64_t spacing =
        ckpt_every > 0 ? ckpt_every
                       : std::max<int64_t>(1, (int64_t)std::llround(std::sqrt((double)nsteps)));
    const int64_t C = store_all ? std::max<int64_t>(nsteps, 1)
                                : std::max<int64_t>(1, std::min<int64_t>(spacing, std::max<int64_t>(nsteps, 1)));
    const int64_t nseg = (nsteps + C - 1) / C;
    DevBuf ck, seg, scratch, work, logs, mis, dcells, actl, prom, stat64, fwd, padst, gmap;
    if ((!store_all && (e = ck.alloc((size_t)nseg * 3 * fe * sizeof(T))) != hipSuccess) ||
        (!store_all && (e = seg.alloc((size_t)C * 3 * fe * sizeof(T))) != hipSuccess) ||
        (e = scratch.alloc(3 * fe * sizeof(double))) != hipSuccess ||
        (e = work.alloc((size_t)swe::adjoint_work_arrays() * Npad * sizeof(double) + 256)) != hipSuccess ||
        (e = logs.alloc(2 * (size_t)std::max<int64_t>(nsteps, 1) * sizeof(double))) != hipSuccess ||
        (e = mis.alloc((size_t)std::max<int64_t>(nobs * ng, 1) * sizeof(double))) != hipSuccess ||
        (e = dcells.alloc((size_t)std::max(ng, 1) * sizeof(long long))) != hipSuccess ||
        (e = actl.alloc(sizeof(Ctl))) != hipSuccess ||
        (e = fwd.alloc(6 * fe * sizeof(double))) != hipSuccess ||
        (e = padst.alloc(2 * Npad * sizeof(double))) != hipSuccess ||
        (e = gmap.alloc((size_t)h->P.nx * (size_t)h->P.ny * sizeof(int))) != hipSuccess)
        return fail(h, SWE_ENOMEM, std::string("swe_grad: hipMalloc failed: ") + hip_text(e));
    // FP64 handles keep U* and U^d of every step of a segment when that fits
    // in a third of the free device memory: the segment's recompute then runs
    // the tracing step, and the reverse sweep replays nothing
    // (SWE_GRAD_KEEP=0 in the environment forces the per-step replay)
    DevBuf segtr;
    bool keep = false;
    const char* keep_env = std::getenv("SWE_GRAD_KEEP");
    if (!mixed && !store_all && !(keep_env && keep_env[0] == '0')) {
        size_t freeb = 0, totalb = 0;
        const size_t need = (size_t)C * 6 * fe * sizeof(double);
        if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && need <= freeb / 3)
            keep = segtr.alloc(need) == hipSuccess;
        (void)hipGetLastError();
    }
    // With the kept U* and U^d, the recompute of the segment below runs on a
    // second stream while the reverse sweep marches the present one, each in
    // its own pair of segment buffers (the same bits: the same kernels on the
    // same operands, ordered by events); SWE_GRAD_OVERLAP=0 in the
    // environment runs them one after the other on the handle's stream
    DevBuf seg2, segtr2;
    SideStream side;
    bool overlap = false;
    const char* ovl_env = std::getenv("SWE_GRAD_OVERLAP");
    if (keep && nseg > 1 && !(ovl_env && ovl_env[0] == '0')) {
        size_t freeb = 0, totalb = 0;
        const size_t need = (size_t)C * 6 * fe * sizeof(double);
        overlap = hipMemGetInfo(&freeb, &totalb) == hipSuccess && need <= freeb / 3 &&
                  seg2.alloc((size_t)C * 3 * fe * sizeof(T)) == hipSuccess &&
                  segtr2.alloc(need) == hipSuccess && side.init() == hipSuccess;
        (void)hipGetLastError();
    }
    // FP64 views the reverse sweep works on
    const double* z64 = (const double*)h->z;
    const double* n64 = (const double*)h->n;
    const double* m64 = (const double*)bufB(h, 3);
    if (mixed) {
        if ((e = prom.alloc(3 * fe * sizeof(double))) != hipSuccess ||
            (e = stat64.alloc(3 * fe * sizeof(double))) != hipSuccess)
            return fail(h, SWE_ENOMEM, std::string("swe_grad: hipMalloc failed: ") + hip_text(e));
        double* zz = stat64.d();
        double* nn = stat64.d() + fe;
        double* mm = stat64.d() + 2 * fe;
        const size_t ne = state_elems(h);
        e = swe::launch_promote((const float*)h->z, zz, ne, h->stream);
        if (e == hipSuccess) e = swe::launch_promote((const float*)h->n, nn, ne, h->stream);
        if (e == hipSuccess) e = swe::launch_manning_m<double>(h->P, nn, mm, h->stream);
        z64 = zz;
        n64 = nn;
        m64 = mm;
    }
    if (e == hipSuccess)
        e = swe::launch_pad_static<double>(h->P, z64, m64, padst.d(), padst.d() + Npad, h->stream);
    if (e == hipSuccess && ng > 0)
        e = hipMemcpyAsync(dcells.p, g->cells, (size_t)ng * sizeof(long long),
                           hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = swe::launch_gauge_map(h->P, (const long long*)dcells.p, ng, (int*)gmap.p, h->stream);
    double* dtlog = logs.d();
    double* tlog = logs.d() + std::max<int64_t>(nsteps, 1);
    if (verbose) {
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        std::fprintf(stderr, "swe_grad: %.1f ms: set-up done\n", ms_since(t_start));
    }
    auto slot = [&](void* base, int64_t m, T* U[3]) {
        for (int f = 0; f < 3; ++f) U[f] = (T*)base + ((size_t)m * 3 + f) * fe;
    };
    // the kept trajectory: step k holds U^k, then U*, then U^d
    auto traj_state = [&](int64_t k, int f) { return traj_base + ((size_t)k * 9 + f) * fe; };
    // ---- forward: the run itself, with checkpoints, time steps and misfits
    if (e == hipSuccess) e = begin_call(h, h->stream);
    if constexpr (!mixed) {
        if (store_all && e == hipSuccess) {
            double* S0[3] = {traj_state(0, 0), traj_state(0, 1), traj_state(0, 2)};
            double* A0[3] = {(double*)bufA(h, 0), (double*)bufA(h, 1), (double*)bufA(h, 2)};
            e = copy_state<double>(h, S0, A0);
        }
    }
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        T* cur[3];
        for (int f = 0; f < 3; ++f) cur[f] = (T*)((k & 1) ? bufB(h, f) : bufA(h, f));
        if constexpr (!mixed) {
            if (store_all) {
                // the tracing step from the kept U^k into U^{k+1} (the last
                // into the buffer the step would have written), U* and U^d
                // kept beside it; the handle's control block advances as in
                // swe_run
                T* last = (T*)((k & 1) ? bufA(h, 0) : bufB(h, 0));
                swe::FusedArgs<double> fa;
                fa.P = h->P;
                fa.ctl = h->ctl;
                fa.t_end = INFINITY;
                fa.eta = traj_state(k, 0); fa.qx = traj_state(k, 1); fa.qy = traj_state(k, 2);
                fa.z = (const double*)h->z;
                fa.m = (const double*)bufB(h, 3);
                for (int f = 0; f < 3; ++f) {
                    double* o = k + 1 < nsteps ? traj_state(k + 1, f)
                                               : (double*)((k & 1) ? bufA(h, f) : bufB(h, f));
                    (f == 0 ? fa.eta1 : (f == 1 ? fa.qx1 : fa.qy1)) = o;
                    fa.tus[f] = traj_state(k, 3 + f);
                    fa.tud[f] = traj_state(k, 6 + f);
                }
                swe::fused_part_layout(fa, h->fpart, h->nparts);
                fa.gy = h->gyt;
                fa.H = h->Ht;
                fa.log_dt = dtlog + k;
                fa.log_t = tlog + k;
                const int sig = ((step0 + k) & 1) ? -1 : 1;
                e = swe::launch_fused_trace(fa, sig, h->stream);
                if (e == hipSuccess && ng > 0 && (k + 1) % g->obs_every == 0) {
                    const int64_t row = (k + 1) / g->obs_every - 1;
                    const double* nxt = k + 1 < nsteps ? traj_state(k + 1, 0) : (const double*)last;
                    e = swe::launch_misfit<double>(h->P, nxt, (const double*)h->z,
                                                   (const long long*)dcells.p, ng,
                                                   g->hobs + row * ng, mis.d() + row * ng,
                                                   h->stream);
                }
                continue;
            }
        }
        if (k % C == 0) {
            T* dst[3];
            slot(ck.p, k / C, dst);
            e = copy_state<T>(h, dst, cur);
        }
        if (e == hipSuccess) e = enqueue(h, k, INFINITY, false, dtlog + k, tlog + k);
        if (e == hipSuccess && ng > 0 && (k + 1) % g->obs_every == 0) {
            const int64_t row = (k + 1) / g->obs_every - 1;
            const T* nxt = (const T*)((k & 1) ? bufA(h, 0) : bufB(h, 0));
            e = swe::launch_misfit<T>(h->P, nxt, (const T*)h->z, (const long long*)dcells.p, ng,
                                      g->hobs + row * ng, mis.d() + row * ng, h->stream);
        }
    }
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e != hipSuccess) return hip_fail(h, e, "swe_grad: forward run");
    rc = fill_stats(h, nullptr);
    if (rc) return rc;
    std::vector<double> hdt((size_t)std::max<int64_t>(nsteps, 1)), ht(hdt.size()),
        hm((size_t)std::max<int64_t>(nobs * ng, 1));
    e = hipMemcpyAsync(hdt.data(), dtlog, hdt.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ht.data(), tlog, ht.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hm.data(), mis.p, hm.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_grad: reading the forward logs");
    double J = 0.0;
    for (int64_t k = 0; k < nobs * ng; ++k) J = J + hm[(size_t)k];
    // ---- reverse sweep, segment by segment
    e = hipMemsetAsync(work.p, 0, (size_t)swe::adjoint_work_arrays() * Npad * sizeof(double) + 256,
                       h->stream);
    // the two-wave march's stall word sits after the work arrays
    int* stall = (int*)(work.d() + (size_t)swe::adjoint_work_arrays() * Npad);
    Ctl* rc_ctl = (Ctl*)actl.p;
    double* US = fwd.d();
    double* UD = fwd.d() + 3 * fe;
    swe::AdjointArgs aa;
    aa.P = h->P;
    for (int f = 0; f < 3; ++f) {
        aa.us[f] = US + (size_t)f * fe;
        aa.ud[f] = UD + (size_t)f * fe;
    }
    aa.zp = padst.d();
    aa.mp = padst.d() + Npad;
    aa.nman = n64;
    aa.work = work.d();
    // the reverse step runs as one fused march of two waves per tile that
    // hand rows over through LDS counters (default), the same two waves in
    // step at a barrier (SWE_ADJOINT=barrier in the environment), the
    // one-wave march (SWE_ADJOINT=march1) or the four gather kernels
    // (SWE_ADJOINT=gather); all give the same bits.  SWE_MARCH_SPIN_CAP
    // lowers the bound on the counter waits (tests of the stall report).
    const char* adj_env = std::getenv("SWE_ADJOINT");
    const bool march =
        !(adj_env && std::strcmp(adj_env, "gather") == 0) && swe::adjoint_march_fits(h->P);
    const swe::MarchMode mmode =
        adj_env && std::strcmp(adj_env, "march1") == 0     ? swe::MarchMode::one_wave
        : adj_env && std::strcmp(adj_env, "barrier") == 0 ? swe::MarchMode::barrier
                                                           : swe::MarchMode::flags;
    int spin_cap = swe::kMarchSpinCap;
    if (const char* cap_env = std::getenv("SWE_MARCH_SPIN_CAP"))
        spin_cap = std::max(0, std::min(swe::kMarchSpinCap, std::atoi(cap_env)));
    int march_rows = 0;
    if (march) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) !=
            hipSuccess)
            cus = 0;
        (void)hipGetLastError();
        march_rows = swe::adjoint_march_rows(h->P, cus, overlap ? 3 : 4);
        // SWE_MARCH_ROWS fixes the march's chunk height (a measurement knob;
        // the gradient is the same bits at any height)
        if (const char* mr = std::getenv("SWE_MARCH_ROWS"))
            if (std::atoi(mr) > 0) march_rows = std::min(256, std::atoi(mr));
    }
    if (verbose)
        std::fprintf(stderr,
                     "swe_grad: %.1f ms: forward run of %lld steps done, %lld reverse segments%s\n",
                     ms_since(t_start), (long long)nsteps, (long long)nseg,
                     store_all ? " (trajectory kept)" : "");
    // the states of segment sg recomputed from its checkpoint into the slots
    // at segp (with U* and U^d at segtrp when kept), on stream st
    auto recompute = [&](int64_t sg, void* segp, double* segtrp, hipStream_t st) -> hipError_t {
        hipError_t r = hipSuccess;
        const int64_t s0 = sg * C, s1 = std::min(s0 + C, nsteps);
        if (!store_all) {
            T *U0[3], *CK[3];
            slot(segp, 0, U0);
            slot(ck.p, sg, CK);
            r = copy_state<T>(h, U0, CK, st);
        }
        // the fused kernel's own finalisation carries dt from step to step.
        // (The recompute runs dense: the dry-tile skip leaves a tile unwritten
        // when the previous step skipped it too, which only a pair of
        // alternating buffers tolerates, not a slot per step.)
        if (r == hipSuccess && !store_all && (keep || s1 - s0 > 1))
            r = swe::launch_replay_ctl(h->P, rc_ctl, ht[(size_t)s0], step0 + s0, hdt[(size_t)s0],
                                       st);
        const int64_t srec = store_all ? s0 : (keep ? s1 : s1 - 1);   // steps recomputed
        for (int64_t k = s0; k < srec && r == hipSuccess; ++k) {
            T *Uk[3], *Un[3];
            slot(segp, k - s0, Uk);
            if (k + 1 < s1) {
                slot(segp, k + 1 - s0, Un);
            } else {
                for (int f = 0; f < 3; ++f) Un[f] = (T*)scratch.p + (size_t)f * fe;
            }
            swe::FusedArgs<T> fa;
            fa.P = h->P;
            fa.ctl = rc_ctl;
            fa.t_end = INFINITY;
            fa.eta = Uk[0]; fa.qx = Uk[1]; fa.qy = Uk[2];
            fa.z = (const T*)h->z;
            fa.m = (const T*)bufB(h, 3);
            fa.eta1 = Un[0]; fa.qx1 = Un[1]; fa.qy1 = Un[2];
            swe::fused_part_layout(fa, h->fpart, h->nparts);
            fa.gy = h->gy;
            fa.H = h->H;
            fa.spin_cap = h->spin_cap;
            const int sig = ((step0 + k) & 1) ? -1 : 1;
            if constexpr (!mixed) {
                if (keep) {
                    double* tk = segtrp + (size_t)(k - s0) * 6 * fe;
                    for (int f = 0; f < 3; ++f) {
                        fa.tus[f] = tk + (size_t)f * fe;
                        fa.tud[f] = tk + (size_t)(3 + f) * fe;
                    }
                    fa.gy = h->gyt;
                    fa.H = h->Ht;
                    r = swe::launch_fused_trace(fa, sig, st);
                    continue;
                }
            }
            r = swe::launch_fused<T>(fa, sig, st, h->more_waves, h->split);
        }
        return r;
    };
    // with the overlap, segment sg lives in buffer pair sg & 1 and the side
    // stream runs one segment ahead of the march
    auto seg_of = [&](int64_t sg) { return overlap && (sg & 1) ? seg2.p : seg.p; };
    auto segtr_of = [&](int64_t sg) { return overlap && (sg & 1) ? segtr2.d() : segtr.d(); };
    if (overlap) {
        const int b = (int)((nseg - 1) & 1);
        e = recompute(nseg - 1, seg_of(nseg - 1), segtr_of(nseg - 1), side.s);
        if (e == hipSuccess) e = hipEventRecord(side.done[b], side.s);
    }
    for (int64_t sg = nseg - 1; sg >= 0 && e == hipSuccess; --sg) {
        if (verbose && sg < nseg - 1) {
            e = hipStreamSynchronize(h->stream);
            std::fprintf(stderr, "swe_grad: %.1f ms: reverse segment %lld of %lld done\n",
                         ms_since(t_start), (long long)(nseg - 1 - sg), (long long)nseg);
            if (e != hipSuccess) break;
        }
        const int64_t s0 = sg * C, s1 = std::min(s0 + C, nsteps);
        void* const segp = seg_of(sg);
        double* const segtrp = segtr_of(sg);
        if (overlap) {
            if (sg > 0) {
                // the segment below, into the pair the march of sg + 1 read
                const int nb = (int)((sg - 1) & 1);
                if (side.used[nb]) e = hipStreamWaitEvent(side.s, side.freed[nb], 0);
                if (e == hipSuccess) e = recompute(sg - 1, seg_of(sg - 1), segtr_of(sg - 1), side.s);
                if (e == hipSuccess) e = hipEventRecord(side.done[nb], side.s);
            }
            if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, side.done[sg & 1], 0);
        } else {
            e = recompute(sg, segp, segtrp, h->stream);
        }
        for (int64_t k = s1 - 1; k >= s0 && e == hipSuccess; --k) {
            T* Uk[3];
            if (store_all)
                for (int f = 0; f < 3; ++f) Uk[f] = (T*)traj_state(k, f);
            else
                slot(segp, k - s0, Uk);
            const double* U64[3] = {(const double*)Uk[0], (const double*)Uk[1],
                                    (const double*)Uk[2]};
            if (mixed) {
                for (int f = 0; f < 3 && e == hipSuccess; ++f) {
                    double* d = prom.d() + (size_t)f * fe;
                    e = swe::launch_promote((const float*)Uk[f], d, state_elems(h), h->stream);
                    U64[f] = d;
                }
            }
            if (e != hipSuccess) break;
            // the step's inflow values, evaluated as the forward step's
            // finalisation evaluated them (same expression, same operands)
            const int L = h->P.hydro_len;
            const double* hyt = h->hydro_host.data();
            aa.qin0 = swe::q_inflow_at(hyt, hyt + std::max(0, L), L, ht[(size_t)k]);
            aa.qin1 = swe::q_inflow_at(hyt, hyt + std::max(0, L), L, ht[(size_t)k] + hdt[(size_t)k]);
            const int sigma = ((step0 + k) & 1) ? -1 : 1;
            const double* US_k = US;
            const double* UD_k = UD;
            if (store_all) {
                // U* and U^d were kept by the forward run
                US_k = traj_state(k, 3);
                UD_k = traj_state(k, 6);
            } else if (keep) {
                // U* and U^d were kept by the segment's recompute
                US_k = segtrp + (size_t)(k - s0) * 6 * fe;
                UD_k = US_k + 3 * fe;
            } else {
                // the step once more in FP64 with its known dt, writing U* and U^d
                e = swe::launch_replay_ctl(h->P, rc_ctl, ht[(size_t)k], step0 + k,
                                           hdt[(size_t)k], h->stream);
                if (e != hipSuccess) break;
                double* Sc = scratch.d();
                swe::FusedArgs<double> ta;
                ta.P = h->P;
                ta.ctl = rc_ctl;
                ta.t_end = INFINITY;
                ta.eta = U64[0]; ta.qx = U64[1]; ta.qy = U64[2];
                ta.z = z64;
                ta.m = m64;
                ta.eta1 = Sc; ta.qx1 = Sc + fe; ta.qy1 = Sc + 2 * fe;
                swe::fused_part_layout(ta, h->fpart, h->nparts);
                ta.gy = h->gyt;
                ta.H = h->Ht;
                for (int f = 0; f < 3; ++f) {
                    ta.tus[f] = US + (size_t)f * fe;
                    ta.tud[f] = UD + (size_t)f * fe;
                }
                e = swe::launch_fused_trace(ta, sigma, h->stream);
                if (e != hipSuccess) break;
            }
            for (int f = 0; f < 3; ++f) {
                aa.un[f] = U64[f];
                aa.us[f] = US_k + (size_t)f * fe;
                aa.ud[f] = UD_k + (size_t)f * fe;
            }
            aa.dt = hdt[(size_t)k];
            aa.rx = aa.dt / h->P.dx;
            aa.ry = aa.dt / h->P.dy;
            aa.sigma = sigma;
            const bool obs = ng > 0 && (k + 1) % g->obs_every == 0;
            const double* hrow = obs ? g->hobs + ((k + 1) / g->obs_every - 1) * ng : nullptr;
            if (march) {
                e = swe::launch_adjoint_march(aa, (const int*)gmap.p, hrow, march_rows,
                                              h->stream, mmode, stall, spin_cap);
                // lambda^n and the bed's share are now in the other slot of each pair
                aa.lam_slot = aa.lam_slot == swe::kAdjLamSlot[0] ? swe::kAdjLamSlot[1]
                                                                 : swe::kAdjLamSlot[0];
                aa.azp_slot = aa.azp_slot == swe::kAdjZpSlot[0] ? swe::kAdjZpSlot[1]
                                                                : swe::kAdjZpSlot[0];
            } else {
                e = swe::launch_adjoint_step(aa, (const int*)gmap.p, hrow, h->stream);
            }
        }
        if (overlap && e == hipSuccess) {
            e = hipEventRecord(side.freed[sg & 1], h->stream);
            side.used[sg & 1] = true;
        }
    }
    if (e == hipSuccess && nsteps > 0) e = swe::launch_adjoint_finish(aa, h->stream);
    if (e == hipSuccess)
        e = swe::launch_unpad(h->P, work.d() + (size_t)swe::kAdjGradN * Npad, (double*)dJ_dn, h->stream);
    if (e == hipSuccess)
        e = swe::launch_unpad(h->P, work.d() + (size_t)swe::kAdjGradZ * Npad, (double*)dJ_dz, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_grad: reverse sweep");
    int stalled = 0;
    e = hipMemcpy(&stalled, stall, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "swe_grad: reverse sweep");
    if (stalled)
        return fail(h, SWE_EDEVICE,
                    "swe_grad: a wave of the reverse march stopped waiting for its partner");
    if (verbose) std::fprintf(stderr, "swe_grad: %.1f ms: reverse sweep done\n", ms_since(t_start));
    *loss = J;
    return SWE_OK;
}

// Gauges of a loss over nsteps steps: counts, distinct cells inside the
// grid, observations in device memory.
int check_gauges(swe_handle* h, int64_t nsteps, const swe_gauges* g, const char* who) {
    if (g->ngauge < 0 || g->obs_every < 1)
        return fail(h, SWE_EINVAL, std::string(who) + ": bad gauges");
    const int64_t nobs = nsteps / g->obs_every;
    const int ng = g->ngauge;
    if (ng > 0 && (!g->cells || (nobs > 0 && !g->hobs)))
        return fail(h, SWE_EINVAL, std::string(who) + ": gauge cells or observations missing");
    std::vector<int64_t> cs(g->cells, g->cells + ng);
    std::sort(cs.begin(), cs.end());
    const int64_t ncell = (int64_t)h->P.nx * h->P.ny;
    for (int k = 0; k < ng; ++k)
        if (cs[k] < 0 || cs[k] >= ncell || (k > 0 && cs[k] == cs[k - 1]))
            return fail(h, SWE_EINVAL,
                        std::string(who) + ": gauge cells must be distinct and inside the grid");
    if (ng > 0 && nobs > 0 && !is_device_ptr(g->hobs, h->device))
        return fail(h, SWE_EINVAL, std::string(who) + ": observations must be device memory");
    return SWE_OK;
}

template <typename T>
int loss_impl(swe_handle* h, int64_t nsteps, const swe_gauges* g, double* loss) {
    const int64_t nobs = nsteps / g->obs_every;
    const int ng = g->ngauge;
    DevBuf mis, dcells;
    hipError_t e;
    if ((e = mis.alloc((size_t)std::max<int64_t>(nobs * ng, 1) * sizeof(double))) != hipSuccess ||
        (e = dcells.alloc((size_t)std::max(ng, 1) * sizeof(long long))) != hipSuccess)
        return fail(h, SWE_ENOMEM, std::string("swe_loss: hipMalloc failed: ") + hip_text(e));
    e = ng > 0 ? hipMemcpyAsync(dcells.p, g->cells, (size_t)ng * sizeof(long long),
                                hipMemcpyHostToDevice, h->stream)
               : hipSuccess;
    if (e == hipSuccess) e = begin_call(h, h->stream);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        e = enqueue(h, k, INFINITY, h->path == SWE_PATH_UNFUSED);
        if (e == hipSuccess && ng > 0 && (k + 1) % g->obs_every == 0) {
            const int64_t row = (k + 1) / g->obs_every - 1;
            const T* nxt = (const T*)((k & 1) ? bufA(h, 0) : bufB(h, 0));
            e = swe::launch_misfit<T>(h->P, nxt, (const T*)h->z, (const long long*)dcells.p, ng,
                                      g->hobs + row * ng, mis.d() + row * ng, h->stream);
        }
    }
    if (e == hipSuccess) e = enqueue_copy_back(h);
    if (e != hipSuccess) return hip_fail(h, e, "swe_loss: forward run");
    int rc = fill_stats(h, nullptr);
    if (rc) return rc;
    std::vector<double> hm((size_t)std::max<int64_t>(nobs * ng, 1));
    e = hipMemcpyAsync(hm.data(), mis.p, hm.size() * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "swe_loss: reading the misfits");
    double J = 0.0;   // the order of swe_grad's sum
    for (int64_t k = 0; k < nobs * ng; ++k) J = J + hm[(size_t)k];
    *loss = J;
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_loss(swe_handle* h, int64_t nsteps, const swe_gauges* g, double* loss) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (nsteps < 0 || !g || !loss) return fail(h, SWE_EINVAL, "swe_loss: bad arguments");
    int rc = check_gauges(h, nsteps, g, "swe_loss");
    if (rc) return rc;
    return h->dtype == SWE_F32 ? loss_impl<float>(h, nsteps, g, loss)
                               : loss_impl<double>(h, nsteps, g, loss);
}

int swe_grad(swe_handle* h, int64_t nsteps, const swe_gauges* g, int32_t ckpt_every,
             double* loss, void* dJ_dn, void* dJ_dz) {
    if (!h) return fail(nullptr, SWE_EINVAL, "handle is NULL");
    if (nsteps < 0 || !g || !loss || !dJ_dn || !dJ_dz || ckpt_every < 0)
        return fail(h, SWE_EINVAL, "swe_grad: bad arguments");
    int rc0 = check_gauges(h, nsteps, g, "swe_grad");
    if (rc0) return rc0;
    if (!is_device_ptr(dJ_dn, h->device) || !is_device_ptr(dJ_dz, h->device))
        return fail(h, SWE_EINVAL, "swe_grad: gradients and observations must be device memory");
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = h->dtype == SWE_F32
                       ? grad_impl<float>(h, nsteps, g, ckpt_every, loss, dJ_dn, dJ_dz)
                       : grad_impl<double>(h, nsteps, g, ckpt_every, loss, dJ_dn, dJ_dz);
    const char* verbose_env = std::getenv("SWE_VERBOSE");
    if (verbose_env && verbose_env[0] == '1')
        std::fprintf(stderr, "swe_grad: %.1f ms: returned (scratch freed)\n",
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                         .count());
    return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ ensemble

struct swe_ensemble {
    std::vector<swe_handle*> h;
    int dtype = SWE_F64;
    hipStream_t stream = nullptr;
    int H = 0;
    double args_t_end = -1.0;   // t_end the device argument arrays were built for
    void* args[2] = {nullptr, nullptr};   // FusedArgs per scenario: even (A->B), odd (B->A)
    int* first = nullptr;                 // count + 1 prefix sums of workgroups
    int total = 0;
    int64_t step_host = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_steps = 0;
    std::string err;
};

namespace {

thread_local std::string g_ens_err = "no error";

int efail(swe_ensemble* e, int code, const std::string& msg) {
    if (e)
        e->err = msg;
    else
        g_ens_err = msg;
    return code;
}

template <typename T>
swe::FusedArgs<T> fused_args_of(swe_handle* h, int parity, double t_end) {
    swe::FusedArgs<T> a;
    a.P = h->P;
    a.ctl = h->ctl;
    a.t_end = t_end;
    const int s = parity & 1;
    a.eta = (const T*)(s ? bufB(h, 0) : bufA(h, 0));
    a.qx = (const T*)(s ? bufB(h, 1) : bufA(h, 1));
    a.qy = (const T*)(s ? bufB(h, 2) : bufA(h, 2));
    a.z = (const T*)h->z;
    a.m = (const T*)bufB(h, 3);
    a.eta1 = (T*)(s ? bufA(h, 0) : bufB(h, 0));
    a.qx1 = (T*)(s ? bufA(h, 1) : bufB(h, 1));
    a.qy1 = (T*)(s ? bufA(h, 2) : bufB(h, 2));
    swe::fused_part_layout(a, h->fpart, h->nparts);
    a.gy = h->gy;
    a.H = h->H;
    a.dry = h->dry;
    a.spin_cap = h->spin_cap;
    return a;
}

template <typename T>
hipError_t upload_args(swe_ensemble* e, double t_end) {
    const size_t n = e->h.size();
    for (int parity = 0; parity < 2; ++parity) {
        std::vector<swe::FusedArgs<T>> v(n);
        for (size_t k = 0; k < n; ++k) v[k] = fused_args_of<T>(e->h[k], parity, t_end);
        hipError_t err = hipMemcpy(e->args[parity], v.data(), n * sizeof(swe::FusedArgs<T>),
                                   hipMemcpyHostToDevice);
        if (err != hipSuccess) return err;
    }
    e->args_t_end = t_end;
    return hipSuccess;
}

hipError_t ens_upload(swe_ensemble* e, double t_end) {
    return e->dtype == SWE_F32 ? upload_args<float>(e, t_end) : upload_args<double>(e, t_end);
}

// Give every scenario tile height H and rebuild the workgroup table.
hipError_t ens_set_tile_rows(swe_ensemble* e, int H) {
    std::vector<int> first(e->h.size() + 1, 0);
    for (size_t k = 0; k < e->h.size(); ++k) {
        swe_handle* h = e->h[k];
        h->H = H;
        h->gy = (h->P.ny + H - 1) / H;
        first[k + 1] = first[k] + swe::fused_blocks(h->P.nx, h->P.ny, H);
    }
    e->H = H;
    e->total = first.back();
    hipError_t err = hipMemcpy(e->first, first.data(), first.size() * sizeof(int),
                               hipMemcpyHostToDevice);
    if (err == hipSuccess) err = ens_upload(e, e->args_t_end < 0.0 ? INFINITY : e->args_t_end);
    return err;
}

hipError_t ens_enqueue(swe_ensemble* e, int64_t nsteps) {
    hipError_t err = hipSuccess;
    for (swe_handle* h : e->h)
        if (err == hipSuccess) err = begin_call(h, e->stream);
    const int count = (int)e->h.size();
    bool dry = false;
    for (swe_handle* h : e->h) dry = dry || h->dry != nullptr;
    // one wave per tile: the two-wave step (SWE_ENSEMBLE_SPLIT=1 in the
    // environment, FP32 only) measured slower here, 312 against 228 ms for the
    // 500-step flood ensemble (short tiles), where the 4096^2 grid gains 4-7%
    const char* es = std::getenv("SWE_ENSEMBLE_SPLIT");
    const bool split = es && std::atoi(es) != 0;
    for (int64_t k = 0; k < nsteps && err == hipSuccess; ++k) {
        const int sigma = ((e->step_host + k) & 1) ? -1 : 1;
        err = e->dtype == SWE_F32
                  ? swe::launch_ensemble<float>((const swe::FusedArgs<float>*)e->args[k & 1],
                                                e->first, count, e->total, sigma, dry, e->stream,
                                                split)
                  : swe::launch_ensemble<double>((const swe::FusedArgs<double>*)e->args[k & 1],
                                                 e->first, count, e->total, sigma, dry, e->stream,
                                                 split);
    }
    for (swe_handle* h : e->h)
        if (err == hipSuccess) err = enqueue_copy_back(h);
    return err;
}

// Restore every scenario to its saved initial state (t = 0, step 0).
hipError_t ens_restore(swe_ensemble* e, const std::vector<void*>& saved) {
    hipError_t err = hipSuccess;
    for (size_t k = 0; k < e->h.size() && err == hipSuccess; ++k) {
        swe_handle* h = e->h[k];
        const size_t n = state_elems(h) * h->elem;
        for (int f = 0; f < 3 && err == hipSuccess; ++f)
            err = hipMemcpyAsync(bufA(h, f), (char*)saved[k] + f * n, n, hipMemcpyDeviceToDevice,
                                 e->stream);
        if (err == hipSuccess) err = swe::launch_init_ctl(h->ctl, 0.0, 0, 0u, 0.0, e->stream);
        if (err == hipSuccess)
            err = h->dtype == SWE_F32
                      ? swe::launch_scan<float>(h->P, h->ctl, INFINITY, (const float*)h->eta,
                                                (const float*)h->qx, (const float*)h->qy,
                                                (const float*)h->z, h->part, h->part + h->nparts,
                                                0, e->stream)
                      : swe::launch_scan<double>(h->P, h->ctl, INFINITY, (const double*)h->eta,
                                                 (const double*)h->qx, (const double*)h->qy,
                                                 (const double*)h->z, h->part,
                                                 h->part + h->nparts, 0, e->stream);
    }
    e->step_host = 0;
    return err;
}

// Time a few steps of the ensemble at each candidate tile height on the
// ensemble itself, keep the fastest, restore the initial states.
int ens_autotune(swe_ensemble* e) {
    static std::map<std::string, int> cache;
    std::string key = std::to_string(e->dtype);
    for (swe_handle* h : e->h) key += "," + std::to_string(h->P.nx) + "x" + std::to_string(h->P.ny);
    auto it = cache.find(key);
    if (it != cache.end()) {
        hipError_t err = ens_set_tile_rows(e, it->second);
        return err == hipSuccess ? SWE_OK : efail(e, SWE_EDEVICE, hip_text(err));
    }
    std::vector<void*> saved(e->h.size(), nullptr);
    auto release = [&]() {
        for (void* p : saved)
            if (p) (void)hipFree(p);
    };
    hipError_t err = hipSuccess;
    for (size_t k = 0; k < e->h.size() && err == hipSuccess; ++k) {
        swe_handle* h = e->h[k];
        const size_t n = state_elems(h) * h->elem;
        err = hipMalloc(&saved[k], 3 * n);
        for (int f = 0; f < 3 && err == hipSuccess; ++f)
            err = hipMemcpyAsync((char*)saved[k] + f * n, bufA(h, f), n, hipMemcpyDeviceToDevice,
                                 e->stream);
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(&ev0);
    if (err == hipSuccess) err = hipEventCreate(&ev1);
    // each height: 2 warm-up steps, then the fastest of 3 timed runs of 4 steps (a single short
    // run picked heights 32 and 64 about equally often on the same ensemble)
    int best = 0;
    float best_ms = 0.0f;
    for (int H : {16, 32, 48, 64, 96, 128}) {
        if (err != hipSuccess) break;
        err = ens_set_tile_rows(e, H);
        if (err == hipSuccess) err = ens_enqueue(e, 2);
        e->step_host += 2;
        float ms_min = 0.0f;
        for (int trial = 0; trial < 3 && err == hipSuccess; ++trial) {
            err = hipEventRecord(ev0, e->stream);
            if (err == hipSuccess) err = ens_enqueue(e, 4);
            e->step_host += 4;
            if (err == hipSuccess) err = hipEventRecord(ev1, e->stream);
            if (err == hipSuccess) err = hipEventSynchronize(ev1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev0, ev1);
            if (err == hipSuccess && (trial == 0 || ms < ms_min)) ms_min = ms;
        }
        if (err == hipSuccess && (best == 0 || ms_min < best_ms)) {
            best = H;
            best_ms = ms_min;
        }
        if (err == hipSuccess) err = ens_restore(e, saved);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    release();
    if (err == hipSuccess) err = ens_set_tile_rows(e, best);
    if (err != hipSuccess) return efail(e, SWE_EDEVICE, std::string("autotuning: ") + hip_text(err));
    cache[key] = best;
    return SWE_OK;
}

}  // namespace

extern "C" {

void swe_ensemble_destroy(swe_ensemble* e) {
    if (!e) return;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    for (swe_handle* h : e->h) swe_destroy(h);
    if (e->args[0]) (void)hipFree(e->args[0]);
    if (e->args[1]) (void)hipFree(e->args[1]);
    if (e->first) (void)hipFree(e->first);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

int swe_ensemble_create(const swe_config* cfgs, int32_t count, int32_t tile_rows,
                        swe_ensemble** out) {
    if (!out) return efail(nullptr, SWE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || count < 1) return efail(nullptr, SWE_EINVAL, "need at least one scenario");
    if (tile_rows < 0) return efail(nullptr, SWE_EINVAL, "tile_rows must be >= 0");
    for (int k = 0; k < count; ++k) {
        if (cfgs[k].dtype != cfgs[0].dtype) return efail(nullptr, SWE_EINVAL, "scenarios mix dtypes");
        if (cfgs[k].path != SWE_PATH_FUSED) return efail(nullptr, SWE_EINVAL, "ensembles use the fused path");
        if (cfgs[k].t0 != 0.0) return efail(nullptr, SWE_EINVAL, "ensemble scenarios start at t0 = 0");
    }
    swe_ensemble* e = new swe_ensemble;
    e->dtype = cfgs[0].dtype;
    hipError_t err = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking);
    if (err != hipSuccess) {
        e->stream = nullptr;
        swe_ensemble_destroy(e);
        return efail(nullptr, SWE_EDEVICE, std::string("hipStreamCreate: ") + hip_text(err));
    }
    for (int k = 0; k < count; ++k) {
        swe_config c = cfgs[k];
        c.stream = e->stream;
        c.tile_rows = tile_rows > 0 ? tile_rows : 16;   // scratch sized for the smallest height
        swe_handle* h = nullptr;
        const int rc = swe_create(&c, &h);
        if (rc != SWE_OK) {
            const std::string msg = std::string("scenario ") + std::to_string(k) + ": " +
                                    swe_last_error(nullptr);
            swe_ensemble_destroy(e);
            return efail(nullptr, rc, msg);
        }
        e->h.push_back(h);
    }
    const size_t asz = e->dtype == SWE_F32 ? sizeof(swe::FusedArgs<float>) : sizeof(swe::FusedArgs<double>);
    if ((err = hipMalloc(&e->args[0], asz * count)) != hipSuccess ||
        (err = hipMalloc(&e->args[1], asz * count)) != hipSuccess ||
        (err = hipMalloc((void**)&e->first, sizeof(int) * (count + 1))) != hipSuccess) {
        swe_ensemble_destroy(e);
        return efail(nullptr, SWE_ENOMEM, std::string("hipMalloc: ") + hip_text(err));
    }
    e->args_t_end = INFINITY;
    if (tile_rows > 0) {
        err = ens_set_tile_rows(e, tile_rows);
        if (err != hipSuccess) {
            swe_ensemble_destroy(e);
            return efail(nullptr, SWE_EDEVICE, hip_text(err));
        }
    } else {
        const int rc = ens_autotune(e);
        if (rc != SWE_OK) {
            const std::string msg = e->err;
            swe_ensemble_destroy(e);
            return efail(nullptr, rc, msg);
        }
    }
    *out = e;
    return SWE_OK;
}

int swe_ensemble_run(swe_ensemble* e, int64_t nsteps, double t_end) {
    if (!e) return efail(nullptr, SWE_EINVAL, "ensemble is NULL");
    if (nsteps < 0 || std::isnan(t_end)) return efail(e, SWE_EINVAL, "bad nsteps or t_end");
    hipError_t err = hipSuccess;
    if (t_end != e->args_t_end) {
        err = hipStreamSynchronize(e->stream);
        if (err == hipSuccess) err = ens_upload(e, t_end);
    }
    if (err == hipSuccess) err = ens_enqueue(e, nsteps);
    if (err != hipSuccess) return efail(e, SWE_EDEVICE, std::string("swe_ensemble_run: ") + hip_text(err));
    e->step_host += nsteps;
    return SWE_OK;
}

int swe_ensemble_capture(swe_ensemble* e, int64_t nsteps) {
    if (!e) return efail(nullptr, SWE_EINVAL, "ensemble is NULL");
    if (nsteps < 0 || (nsteps & 1)) return efail(e, SWE_EINVAL, "capture needs an even step count");
    if (e->step_host & 1) return efail(e, SWE_EINVAL, "capture must start on an even step");
    hipError_t err = hipStreamSynchronize(e->stream);
    if (err == hipSuccess && e->args_t_end != INFINITY) err = ens_upload(e, INFINITY);
    if (e->exec) {
        (void)hipGraphExecDestroy(e->exec);
        e->exec = nullptr;
    }
    if (e->graph) {
        (void)hipGraphDestroy(e->graph);
        e->graph = nullptr;
    }
    if (err == hipSuccess) err = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
        const hipError_t enq = ens_enqueue(e, nsteps);
        err = hipStreamEndCapture(e->stream, &e->graph);
        if (enq != hipSuccess) err = enq;
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
    if (err != hipSuccess) return efail(e, SWE_EDEVICE, std::string("graph capture: ") + hip_text(err));
    e->graph_steps = nsteps;
    return SWE_OK;
}

int swe_ensemble_replay(swe_ensemble* e) {
    if (!e) return efail(nullptr, SWE_EINVAL, "ensemble is NULL");
    if (!e->exec) return efail(e, SWE_EINVAL, "nothing captured");
    if (e->step_host & 1) return efail(e, SWE_EINVAL, "replay must start on an even step");
    hipError_t err = hipGraphLaunch(e->exec, e->stream);
    if (err != hipSuccess) return efail(e, SWE_EDEVICE, std::string("hipGraphLaunch: ") + hip_text(err));
    e->step_host += e->graph_steps;
    return SWE_OK;
}

int swe_ensemble_stats(swe_ensemble* e, swe_stats* out) {
    if (!e) return efail(nullptr, SWE_EINVAL, "ensemble is NULL");
    hipError_t err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) return efail(e, SWE_EDEVICE, hip_text(err));
    int worst = SWE_OK;
    for (size_t k = 0; k < e->h.size(); ++k) {
        const int rc = fill_stats(e->h[k], out ? out + k : nullptr);
        if (rc != SWE_OK) {
            worst = rc;
            e->err = "scenario " + std::to_string(k) + ": " + e->h[k]->err;
        }
    }
    return worst;
}

int32_t swe_ensemble_tile_rows(const swe_ensemble* e) { return e ? e->H : 0; }

const char* swe_ensemble_last_error(const swe_ensemble* e) {
    return e ? e->err.c_str() : g_ens_err.c_str();
}

const char* swe_last_error(const swe_handle* h) {
    return h ? h->err.c_str() : g_create_err.c_str();
}

int swe_probe_stream(const void* const* in, void* const* out, size_t bytes, int nontemporal,
                     void* stream) {
    if (!in || !out) return fail(nullptr, SWE_EINVAL, "swe_probe_stream: NULL array list");
    for (int k = 0; k < 5; ++k)
        if (!in[k] || ((uintptr_t)in[k] % 16))
            return fail(nullptr, SWE_EINVAL, "swe_probe_stream: inputs must be 16-byte aligned");
    for (int k = 0; k < 3; ++k)
        if (!out[k] || ((uintptr_t)out[k] % 16))
            return fail(nullptr, SWE_EINVAL, "swe_probe_stream: outputs must be 16-byte aligned");
    if (bytes % 16) return fail(nullptr, SWE_EINVAL, "swe_probe_stream: bytes must be a multiple of 16");
    hipError_t e = swe::launch_stream8(in, out, bytes / 16, nontemporal != 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "swe_probe_stream");
    return SWE_OK;
}

int swe_probe_march(const void* const* in, void* const* out, int32_t nx, int32_t ny,
                    int64_t pitch, int32_t elem_bytes, int32_t rows, void* stream) {
    if (!in || !out) return fail(nullptr, SWE_EINVAL, "swe_probe_march: NULL array list");
    if (elem_bytes != 4 && elem_bytes != 8)
        return fail(nullptr, SWE_EINVAL, "swe_probe_march: elem_bytes must be 4 or 8");
    if (nx < 1 || ny < 1 || pitch < nx || (long long)ny * pitch > (1ll << 31))
        return fail(nullptr, SWE_EINVAL, "swe_probe_march: need 1 <= nx <= pitch, ny >= 1, ny*pitch <= 2^31");
    if (rows < 0) return fail(nullptr, SWE_EINVAL, "swe_probe_march: rows must be >= 0");
    swe::ProbeMarchArgs a;
    for (int k = 0; k < 5; ++k) {
        if (!in[k] || ((uintptr_t)in[k] % elem_bytes))
            return fail(nullptr, SWE_EINVAL, "swe_probe_march: inputs must be non-NULL and aligned");
        a.in[k] = in[k];
    }
    for (int k = 0; k < 3; ++k) {
        if (!out[k] || ((uintptr_t)out[k] % elem_bytes))
            return fail(nullptr, SWE_EINVAL, "swe_probe_march: outputs must be non-NULL and aligned");
        a.out[k] = out[k];
    }
    int H = rows;
    if (H == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        H = swe::probe_march_rows(elem_bytes, nx, ny, cus);
    }
    const long long gy = ((long long)ny + H - 1) / H;
    if ((long long)swe::fused_strips(nx) * gy > (1ll << 30))
        return fail(nullptr, SWE_EINVAL, "swe_probe_march: too many tiles");
    a.nx = nx;
    a.ny = ny;
    a.H = H;
    a.gy = (int)gy;
    a.pitch = pitch;
    hipError_t e = swe::launch_probe_march(a, elem_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "swe_probe_march");
    return H;
}

int swe_probe_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || (bytes % 16) || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(nullptr, SWE_EINVAL, "swe_probe_copy: pointers must be 16-byte aligned and bytes a multiple of 16");
    hipError_t e = swe::launch_copy16(dst, src, bytes / 16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "swe_probe_copy");
    return SWE_OK;
}

}  // extern "C"
