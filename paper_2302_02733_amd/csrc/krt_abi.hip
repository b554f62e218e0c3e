// C ABI of the polarized Kerr ray tracer (see include/krt.h): host-side
// validation, context and scratch management, kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "krt.h"
#include "krt_kernels.hpp"
#include "krt_validate.hpp"

using namespace krt;

struct krt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    bool units_set = false;
    krt_units units{};
    int model = -1;
    krt_adaf adaf{};
    krt_snapshot_desc snap{};
    const double* snap_prims = nullptr;
    const float* snap_prims_f = nullptr;
    // layout-1 snapshots are read through a library-owned layout-0 copy
    void* snap_copy = nullptr;
    size_t snap_copy_bytes = 0;
    // start values of the MKS inversion for the snapshot's hslope
    double* x2tab = nullptr;
    int precision = KRT_PRECISION_FP64;
    double* btab = nullptr;
    // wave-synchronous path store
    double* pool = nullptr;
    size_t pool_bytes = 0;
    int pool_cap = 0;
    int pool_blocks = 0;       // blocks the store holds slices for
    int launch_blocks = 0;     // blocks of the current mode's launch (<= pool_blocks)
    // paged extension of the wave store
    double* chunk_pool = nullptr;
    unsigned* chunk_flags = nullptr;
    int nchunks = 0;
    int chunk_cap = 0;
    // long-ray store
    double* long_pool = nullptr;
    size_t long_bytes = 0;
    int long_slots = 0;
    int long_max_steps = -1;
    int32_t* overflow_list = nullptr;
    int32_t* overflow_inst = nullptr;
    size_t overflow_cap = 0;
    // pixel list of the measurement probe
    int32_t* probe_dev = nullptr;
    size_t probe_cap = 0;

    // launch configuration (tile shape, grid, slice size)
    krt_launch_config cfg{sizeof(krt_launch_config), 8, 0, 0, 1};
    // batch descriptors: device copy and pinned staging
    void* batch_dev = nullptr;
    size_t batch_dev_bytes = 0;
    void* batch_host = nullptr;
    size_t batch_host_bytes = 0;
    // counters: [0] tile queue, [1] overflow count (unsigned); then 10 x u64;
    // then the 8 sector queues
    unsigned* work = nullptr;
    double* red_partial = nullptr;
    double* host_buf = nullptr;  // pinned, 16 doubles
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    // nonthermal electrons: synchrotron-function table (built on first use)
    double* syntab = nullptr;
    // surrogate: FP32 master parameters, Adam moments, normalisation, packed form
    float* mlp_P = nullptr;
    float* mlp_m = nullptr;
    float* mlp_v = nullptr;
    double* mlp_norm = nullptr;
    MlpPacked* mlp_packed = nullptr;
    bool mlp_ready = false;
    // plain-mode tile order (centre first) for the last image shape
    int* tile_order = nullptr;
    int tile_order_cap = 0;
    int tile_order_key[4] = {0, 0, 0, 0};   // tiles_x, tiles_y, tile_w, sectors
    int electrons = KRT_ELECTRONS_THERMAL;
    double kappa = 5.0;
    std::string err;
};

// Device scratch of the allocation-free reduction (see kScratchDoubles below):
// one copy per device, alive until the process ends.
static __device__ __align__(256) double scratch[1024 * 9 + 16];

namespace {

constexpr int kSectors = 8;   // XCDs of the device: one image sector each
constexpr int kWorkWords = 2 + 2 * 10 + kSectors;
constexpr int kRedBlocks = 1024;

// Scratch of the allocation-free reduction (krt_reduce_noalloc): the block
// partials of reduce_partial (9 doubles for each of at most kRedBlocks blocks)
// and the five results, 73.9 KB per device whatever the image size.  Host code
// never uses the array's name as an address: each device's address comes from
// hipGetSymbolAddress at context creation (kept in g_scratch_dev).
constexpr size_t kScratchDoubles = (size_t)kRedBlocks * 9 + 16;
static_assert(sizeof(scratch) == kScratchDoubles * sizeof(double), "scratch size");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Looks up this device's copy of `scratch` once (the device must be current).
hipError_t resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return hipSuccess;   // the entry point refuses such devices
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_dev[device] = static_cast<double*>(p);
    return e;
}

krt_status fail(krt_ctx* ctx, krt_status code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

krt_status hip_fail(krt_ctx* ctx, hipError_t e, const char* what) {
    return fail(ctx, KRT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define KRT_HIP(ctx, call)                                          \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);    \
    } while (0)

using krt_host::check_camera;
using krt_host::finite_all;
using krt_host::horizon;
using krt_host::isco;

CameraDesc camera_desc(const krt_camera* c) {
    CameraDesc d;
    d.a = c->a;
    d.m = (double)c->mass_factor;
    d.r_cam = c->r_cam;
    d.th = c->incl_deg * kPi / 180.0;
    d.ph = c->phi_deg * kPi / 180.0;
    d.fov_x = c->fov_x;
    d.fov_y = c->fov_y;
    d.freq = c->freq_hz;
    d.nx = c->nx;
    d.ny = c->ny;
    d.jitter = c->jitter;
    d.seed = c->seed;
    return d;
}

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}

void fill_f32(krt_ctx* ctx, double nu, TraceArgs& A);

TraceArgs base_args(krt_ctx* ctx, const krt_camera* cam) {
    TraceArgs A;
    std::memset(&A, 0, sizeof(A));
    A.cam = camera_desc(cam);
    A.eps = cam->eps;
    A.r_stop = cam->mass_factor == 0 ? 1e-6 : 1.05 * horizon(cam->a, 1.0);
    A.L_cm = ctx->units_set ? kG * ctx->units.M_bh_g / (kC * kC) : 0.0;
    A.fac0 = A.L_cm / cam->freq_hz;
    A.max_steps = cam->max_steps;
    A.model = ctx->model < 0 ? kModelAdaf : ctx->model;
    if (ctx->model == kModelSnapshot) {
        const krt_snapshot_desc& d = ctx->snap;
        const double L = A.L_cm;
        A.snap.prims = ctx->snap_prims;
        A.snap.prims_f = ctx->snap_prims_f;
        A.snap.n1 = d.n1;
        A.snap.n2 = d.n2;
        A.snap.n3 = d.n3;
        A.snap.x1s = d.x1_start;
        A.snap.dx1 = d.dx1;
        A.snap.x2s = d.x2_start;
        A.snap.dx2 = d.dx2;
        A.snap.x3s = d.x3_start;
        A.snap.dx3 = d.dx3;
        A.snap.idx1 = 1.0 / d.dx1;   // dx > 0 (checked)
        A.snap.idx2 = 1.0 / d.dx2;
        A.snap.idx3 = 1.0 / d.dx3;
        A.snap.in3 = 1.0 / d.n3;     // n3 > 0 (checked)
        A.snap.h = d.hslope;
        A.snap.gam = d.gamma_ad;
        A.snap.rho_unit = L > 0.0 ? d.M_unit_g / (L * L * L) : 0.0;
        A.snap.B_unit = kC * std::sqrt(4.0 * kPi * A.snap.rho_unit);
        A.snap.Rhigh = d.R_high;
        A.snap.Rlow = d.R_low;
        A.snap.sigma_cut = d.sigma_cut;
        A.snap.rmax = d.r_emit_max;
        A.snap.x2tab = ctx->x2tab;
    }
    A.adaf.n0 = ctx->adaf.n0_cgs;
    A.adaf.T0 = ctx->adaf.T0_K;
    A.adaf.beta = ctx->adaf.beta;
    A.adaf.h = ctx->adaf.h_over_r;
    A.adaf.ibeta = 1.0 / ctx->adaf.beta;                                  // beta > 0 (checked)
    A.adaf.i2h2 = 1.0 / (2.0 * ctx->adaf.h_over_r * ctx->adaf.h_over_r);   // h > 0 (checked)
    A.adaf.risco = isco(cam->a);
    A.btab = ctx->btab;
    fill_f32(ctx, cam->freq_hz, A);
    const int tw = ctx->cfg.tile_w;
    A.tile_w = tw;
    A.tiles_x = (cam->nx + tw - 1) / tw;
    A.nbatch = A.tiles_x * ((cam->ny + 64 / tw - 1) / (64 / tw));
    A.queue = ctx->work;
    A.squeue = ctx->work + 2 + 2 * 10;
    A.nsec = 1;
    A.overflow_count = ctx->work + 1;
    A.counters = reinterpret_cast<unsigned long long*>(ctx->work + 2);
    return A;
}

// Constants of the FP32 transfer operators for camera frequency nu and the
// model parameters already in A, folded in FP64.
void fill_f32(krt_ctx* ctx, double nu, TraceArgs& A) {
    {
        F32Consts& C = A.f32;
        const double L = A.L_cm, e2 = kE * kE;
        C.a = (float)A.cam.a;
        C.m = (float)A.cam.m;
        C.cJ = (float)(e2 * nu / (2.0 * std::sqrt(3.0) * kC));
        C.cRV = (float)(2.0 * e2 / (kME * kC * nu * nu));
        C.cRQ = (float)(e2 / (kME * kC * nu * nu * nu));
        C.cHnu = (float)(kH * nu / (kME * kC * kC));
        C.cBnu = (float)(2.0 * kH * nu * nu * nu / (kC * kC));
        C.cSeq = (float)(kIScale * 2.0 * kH / (kC * kC));
        C.nu_cam = (float)nu;
        C.L = (float)L;
        C.n0 = (float)A.adaf.n0;
        C.thr = (float)(kKB * A.adaf.T0 / (kME * kC * kC));
        C.cB2 = (float)(A.adaf.beta > 0.0 ? 8.0 * kPi * kMP * kC * kC / (6.0 * A.adaf.beta) : 0.0);
        C.ih2 = (float)(A.adaf.h > 0.0 ? 1.0 / (2.0 * A.adaf.h * A.adaf.h) : 0.0);
        C.risco = (float)A.adaf.risco;
        if (ctx->model == kModelSnapshot) {
            C.x1s = (float)A.snap.x1s;
            C.idx1 = (float)(1.0 / A.snap.dx1);
            C.x2s = (float)A.snap.x2s;
            C.idx2 = (float)(1.0 / A.snap.dx2);
            C.hh = (float)(0.5 * (1.0 - A.snap.h));
            C.gm1 = (float)(A.snap.gam - 1.0);
            C.ne_unit = (float)(A.snap.rho_unit / (kMP + kME));
            C.B_unit = (float)A.snap.B_unit;
            C.Rhigh = (float)A.snap.Rhigh;
            C.Rlow = (float)A.snap.Rlow;
            C.sigma_cut = (float)A.snap.sigma_cut;
            C.rmax = (float)A.snap.rmax;
            C.mpme = (float)(kMP / kME);
        }
    }
}

// Sizes the wave-synchronous store: one slice of `cap` points for every
// wavefront of the persistent grid of the kernel about to run (as many blocks
// as fit on the device, within the KRT_POOL_GB budget).  The store only grows.
template <int kMode>
krt_status ensure_pool(krt_ctx* ctx, bool batch = false) {
    const int cap = ctx->cfg.path_cap > 0 ? ctx->cfg.path_cap : env_int("KRT_PATH_CAP", 8192);
    const double budget_gb = (double)env_int("KRT_POOL_GB", 96);
    int per_cu = 0;
    if (batch) {
        if constexpr (kMode == kModeF64 || kMode == kModeF32)
            KRT_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_batch<kMode>, 256, 0));
    } else {
        KRT_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_waves<kMode>, 256, 0));
    }
    if (per_cu < 1) per_cu = 1;
    if (ctx->cfg.blocks_per_cu > 0 && ctx->cfg.blocks_per_cu < per_cu) per_cu = ctx->cfg.blocks_per_cu;
    int blocks = per_cu * ctx->cu_count;
    const size_t per_block = (size_t)4 * 64 * cap * kPointDoubles * sizeof(double);
    const size_t budget = (size_t)(budget_gb * 1073741824.0);
    if ((size_t)blocks * per_block > budget) blocks = (int)(budget / per_block);
    if (blocks < 1) return fail(ctx, KRT_E_NOMEM, "path store budget too small");
    ctx->launch_blocks = blocks;
    if (ctx->pool && ctx->pool_cap == cap && ctx->pool_blocks >= blocks) {
        ctx->launch_blocks = blocks;
        return KRT_OK;
    }
    const size_t need = (size_t)blocks * per_block;
    if (ctx->pool) {
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        KRT_HIP(ctx, hipFree(ctx->pool));
        ctx->pool = nullptr;
    }
    if (hipMalloc(&ctx->pool, need) != hipSuccess) {
        ctx->pool = nullptr;
        (void)hipGetLastError();
        return fail(ctx, KRT_E_NOMEM, "cannot allocate the path store");
    }
    ctx->pool_bytes = need;
    ctx->pool_cap = cap;
    ctx->pool_blocks = blocks;
    ctx->launch_blocks = blocks;
    return KRT_OK;
}

// Chunks of the paged path store (KRT_CHUNKS, default 64, of cap x 64 lanes
// x 64 B: 2 GiB at cap 8192), lent to waves whose rays outgrow their slice.
krt_status ensure_chunks(krt_ctx* ctx) {
    const int cap = ctx->pool_cap;
    int count = env_int("KRT_CHUNKS", 64);
    if (count < 0) count = 0;
    if (count > 4096) count = 4096;
    if (ctx->chunk_cap == cap && ctx->nchunks == count && (count == 0 || ctx->chunk_pool)) return KRT_OK;
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->chunk_pool) KRT_HIP(ctx, hipFree(ctx->chunk_pool));
    if (ctx->chunk_flags) KRT_HIP(ctx, hipFree(ctx->chunk_flags));
    ctx->chunk_pool = nullptr;
    ctx->chunk_flags = nullptr;
    ctx->nchunks = 0;
    ctx->chunk_cap = cap;
    if (count == 0) return KRT_OK;
    const size_t bytes = (size_t)count * cap * 64 * kPointDoubles * sizeof(double);
    if (hipMalloc(&ctx->chunk_pool, bytes) != hipSuccess ||
        hipMalloc(&ctx->chunk_flags, (size_t)count * sizeof(unsigned)) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->chunk_pool) (void)hipFree(ctx->chunk_pool);
        ctx->chunk_pool = nullptr;
        ctx->chunk_flags = nullptr;
        return fail(ctx, KRT_E_NOMEM, "cannot allocate the path chunks");
    }
    ctx->nchunks = count;
    return KRT_OK;
}

krt_status ensure_long(krt_ctx* ctx, int max_steps, size_t npix) {
    if (ctx->long_pool == nullptr || ctx->long_max_steps != max_steps) {
        if (ctx->long_pool) {
            KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
            KRT_HIP(ctx, hipFree(ctx->long_pool));
            ctx->long_pool = nullptr;
        }
        const size_t per = (size_t)(max_steps + 1) * kPointDoubles * sizeof(double);
        int slots = 1024;
        while (slots > 64 && (size_t)slots * per > ((size_t)4 << 30)) slots /= 2;
        if (hipMalloc(&ctx->long_pool, (size_t)slots * per) != hipSuccess) {
            ctx->long_pool = nullptr;
            (void)hipGetLastError();
            return fail(ctx, KRT_E_NOMEM, "cannot allocate the long-ray store");
        }
        ctx->long_slots = slots;
        ctx->long_max_steps = max_steps;
        ctx->long_bytes = (size_t)slots * per;
    }
    if (ctx->overflow_cap < npix) {
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->overflow_list) KRT_HIP(ctx, hipFree(ctx->overflow_list));
        if (ctx->overflow_inst) KRT_HIP(ctx, hipFree(ctx->overflow_inst));
        ctx->overflow_list = nullptr;
        ctx->overflow_inst = nullptr;
        ctx->overflow_cap = 0;
        if (hipMalloc(&ctx->overflow_list, npix * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&ctx->overflow_inst, npix * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            if (ctx->overflow_list) (void)hipFree(ctx->overflow_list);
            ctx->overflow_list = nullptr;
            ctx->overflow_inst = nullptr;
            return fail(ctx, KRT_E_NOMEM, "cannot allocate the overflow list");
        }
        ctx->overflow_cap = npix;
    }
    return KRT_OK;
}

krt_status fill_stats(krt_ctx* ctx, int64_t rays, krt_stats* s) {
    KRT_HIP(ctx, hipMemcpyAsync(ctx->host_buf, ctx->work + 2, 10 * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned long long* c = reinterpret_cast<const unsigned long long*>(ctx->host_buf);
    s->struct_size = sizeof(krt_stats);
    s->rays = rays;
    s->total_steps = (int64_t)c[0];
    for (int k = 0; k < 5; ++k) s->status_count[k] = (int64_t)c[1 + k];
    s->max_steps_seen = (int32_t)c[6];
    s->long_rays = (int64_t)c[7];
    s->surrogate_points = (int64_t)c[8];
    s->exact_points = (int64_t)c[9];
    float t0 = 0.0f, t1 = 0.0f;
    KRT_HIP(ctx, hipEventElapsedTime(&t0, ctx->ev[0], ctx->ev[1]));
    KRT_HIP(ctx, hipEventElapsedTime(&t1, ctx->ev[1], ctx->ev[2]));
    s->kernel_ms[0] = t0;
    s->kernel_ms[1] = t1;
    return KRT_OK;
}

krt_status check_ready(krt_ctx* ctx, const krt_camera* cam) {
    if (!ctx) return KRT_E_INVAL;
    const std::string m = check_camera(cam);
    if (!m.empty()) return fail(ctx, KRT_E_INVAL, m);
    if (!ctx->units_set) return fail(ctx, KRT_E_STATE, "units not set");
    if (ctx->model < 0) return fail(ctx, KRT_E_STATE, "no plasma model set");
    return KRT_OK;
}


// Queue order of the plain tracer's tiles: by distance of the tile centre
// from the image centre, nearest first.  Rays near the shadow's edge (near
// the centre) are the longest; starting them first leaves cheap tiles for
// the end of the launch (on the 1024^2 ADAF image a simulated schedule of
// 2048 waves ends 21% after the ideal in row-major order and 5.5% centre
// first).  Rebuilt when the image shape changes; synchronous upload.
krt_status ensure_tile_order(krt_ctx* ctx, int tiles_x, int tiles_y, int tile_w, const int** out,
                             int* nsec) {
    *out = nullptr;
    *nsec = 1;
    if (ctx->cfg.order != 1 && ctx->cfg.order != 2) return KRT_OK;
    const int sectors = ctx->cfg.order == 2 ? kSectors : 1;
    const int n = tiles_x * tiles_y;
    const int head = sectors > 1 ? sectors + 1 : 0;
    if (ctx->tile_order && ctx->tile_order_key[0] == tiles_x && ctx->tile_order_key[1] == tiles_y &&
        ctx->tile_order_key[2] == tile_w && ctx->tile_order_key[3] == sectors) {
        *out = ctx->tile_order;
        *nsec = sectors;
        return KRT_OK;
    }
    if (n + head > ctx->tile_order_cap) {
        if (ctx->tile_order) {
            KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
            KRT_HIP(ctx, hipFree(ctx->tile_order));
            ctx->tile_order = nullptr;
        }
        if (hipMalloc(&ctx->tile_order, (size_t)(n + kSectors + 1) * sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->tile_order = nullptr;
            ctx->tile_order_cap = 0;
            return fail(ctx, KRT_E_NOMEM, "cannot allocate the tile order");
        }
        ctx->tile_order_cap = n + kSectors + 1;
    }
    // centre-first: tiles by distance of their centre from the image centre;
    // with sectors, first by the 45-degree sector of the image around its
    // centre that holds the tile centre
    std::vector<int> ord(n), sec(n, 0);
    std::vector<double> d2(n);
    const int th = 64 / tile_w;
    const double cx = 0.5 * tiles_x * tile_w, cy = 0.5 * tiles_y * th;
    for (int t = 0; t < n; ++t) {
        ord[t] = t;
        const double x = ((t % tiles_x) + 0.5) * tile_w - cx, y = ((t / tiles_x) + 0.5) * th - cy;
        d2[t] = x * x + y * y;
        if (sectors > 1) {
            const double ang = std::atan2(y, x) + kPi;   // [0, 2 pi]
            int s = (int)(ang * (sectors / (2.0 * kPi)));
            sec[t] = s < 0 ? 0 : (s >= sectors ? sectors - 1 : s);
        }
    }
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return sec[a] != sec[b] ? sec[a] < sec[b] : d2[a] < d2[b]; });
    std::vector<int> buf(head + n);
    if (sectors > 1) {
        std::vector<int> cnt(sectors, 0);
        for (int t = 0; t < n; ++t) ++cnt[sec[t]];
        buf[0] = 0;
        for (int s = 0; s < sectors; ++s) buf[s + 1] = buf[s] + cnt[s];
    }
    for (int k = 0; k < n; ++k) buf[head + k] = ord[k];
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    KRT_HIP(ctx, hipMemcpy(ctx->tile_order, buf.data(), buf.size() * sizeof(int), hipMemcpyHostToDevice));
    ctx->tile_order_key[0] = tiles_x;
    ctx->tile_order_key[1] = tiles_y;
    ctx->tile_order_key[2] = tile_w;
    ctx->tile_order_key[3] = sectors;
    *out = ctx->tile_order;
    *nsec = sectors;
    return KRT_OK;
}

// Synchrotron-function table of the nonthermal module, built on first use.
krt_status ensure_syntab(krt_ctx* ctx) {
    if (ctx->syntab) return KRT_OK;
    double* vals = nullptr;
    double* tab = nullptr;
    if (hipMalloc(&vals, (size_t)kSynPanels * kSynCoef * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&tab, (size_t)kSynTab * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        if (vals) (void)hipFree(vals);
        return fail(ctx, KRT_E_NOMEM, "cannot allocate the synchrotron table");
    }
    const int nn = kSynPanels * kSynCoef;
    hipLaunchKernelGGL(syn_table_nodes, dim3((nn + 127) / 128), dim3(128), 0, ctx->stream, vals);
    hipLaunchKernelGGL(syn_table_coefs, dim3((kSynTab + 127) / 128), dim3(128), 0, ctx->stream, vals, tab);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(vals);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(tab);
        return hip_fail(ctx, e, "synchrotron table");
    }
    ctx->syntab = tab;
    return KRT_OK;
}

krt_status ensure_mlp(krt_ctx* ctx) {
    if (ctx->mlp_P) return KRT_OK;
    if (hipMalloc(&ctx->mlp_P, kMlpParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&ctx->mlp_m, kMlpParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&ctx->mlp_v, kMlpParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&ctx->mlp_norm, kNormLen * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx->mlp_packed, sizeof(MlpPacked)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KRT_E_NOMEM, "cannot allocate the surrogate's parameters");
    }
    return KRT_OK;
}

krt_status mlp_repack(krt_ctx* ctx) {
    hipLaunchKernelGGL(mlp_pack, dim3(1), dim3(256), 0, ctx->stream, ctx->mlp_P, ctx->mlp_norm, ctx->mlp_packed);
    KRT_HIP(ctx, hipGetLastError());
    ctx->mlp_ready = true;
    return KRT_OK;
}

uint64_t splitmix_next(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One pass of the training kernel over samples [first, first + count) of the
// prepared set, partials into gpart / lpart; returns the number of blocks.
int mlp_pass(krt_ctx* ctx, const float* feat, const float* targ, int64_t n, int64_t first, int64_t count,
             bool permute, uint64_t a, uint64_t c, float* gpart, double* lpart) {
    MlpTrainArgs A;
    A.P = ctx->mlp_P;
    A.feat = feat;
    A.targ = targ;
    A.n = n;
    A.first = first;
    A.count = count;
    A.perm_a = a;
    A.perm_c = c;
    A.permute = permute ? 1 : 0;
    A.inv_norm = (float)(1.0 / (8.0 * (double)count));
    A.gpart = gpart;
    A.lpart = lpart;
    const int blocks = (int)((count + kTrainTile - 1) / kTrainTile);
    hipLaunchKernelGGL(mlp_train_tile, dim3(blocks), dim3(256), 0, ctx->stream, A);
    return blocks;
}

// Least-squares cubic baseline of log10 I on the set (normal equations summed
// on the device, solved here by Cholesky), and mu = 0, sd = the rms residual.
krt_status mlp_fit_baseline(krt_ctx* ctx, int64_t n, const double* d_in, const double* d_integ) {
    const int blocks = 256;
    double* d_sums = nullptr;
    if (hipMalloc(&d_sums, (size_t)blocks * kFitLen * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KRT_E_NOMEM, "cannot allocate fit sums");
    }
    hipLaunchKernelGGL(mlp_fit_sums, dim3(blocks), dim3(256), 0, ctx->stream, n, d_in, d_integ, d_sums);
    std::vector<double> h((size_t)blocks * kFitLen);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_sums, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                            ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d_sums);
    if (e != hipSuccess) return hip_fail(ctx, e, "baseline fit");
    std::vector<double> S(kFitLen, 0.0);
    for (int b = 0; b < blocks; ++b)
        for (int q = 0; q < kFitLen; ++q) S[q] += h[(size_t)b * kFitLen + q];
    const int T = kPolyTerms;
    // Cholesky of M^T M
    std::vector<double> L(T * T, 0.0);
    for (int i = 0; i < T; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = S[i * T + j];
            for (int k = 0; k < j; ++k) v -= L[i * T + k] * L[j * T + k];
            if (i == j) {
                if (!(v > 0.0)) return fail(ctx, KRT_E_INVAL, "baseline fit is singular (too few samples?)");
                L[i * T + i] = std::sqrt(v);
            } else {
                L[i * T + j] = v / L[j * T + j];
            }
        }
    std::vector<double> norm(kNormLen, 0.0);
    for (int o = 0; o < 8; ++o) {
        double z[kPolyTerms], c[kPolyTerms];
        for (int i = 0; i < T; ++i) {
            double v = S[T * T + i * 8 + o];
            for (int k = 0; k < i; ++k) v -= L[i * T + k] * z[k];
            z[i] = v / L[i * T + i];
        }
        for (int i = T - 1; i >= 0; --i) {
            double v = z[i];
            for (int k = i + 1; k < T; ++k) v -= L[k * T + i] * c[k];
            c[i] = v / L[i * T + i];
        }
        // residual sum of squares: y^T y - c^T M^T y
        double rss = S[T * T + T * 8 + o];
        for (int i = 0; i < T; ++i) rss -= c[i] * S[T * T + i * 8 + o];
        norm[o] = 0.0;
        norm[8 + o] = std::sqrt(std::max(rss / (double)n, 1e-30));
        for (int i = 0; i < T; ++i) norm[16 + o * T + i] = c[i];
    }
    KRT_HIP(ctx, hipMemcpyAsync(ctx->mlp_norm, norm.data(), kNormLen * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KRT_OK;
}

struct MlpScratch {
    float* feat = nullptr;
    float* targ = nullptr;
    float* gpart = nullptr;
    double* lpart = nullptr;
    double* loss = nullptr;
    ~MlpScratch() {
        if (feat) (void)hipFree(feat);
        if (targ) (void)hipFree(targ);
        if (gpart) (void)hipFree(gpart);
        if (lpart) (void)hipFree(lpart);
        if (loss) (void)hipFree(loss);
    }
};

krt_status mlp_scratch(krt_ctx* ctx, MlpScratch& S, int64_t n, int64_t max_batch) {
    const int64_t blocks = (max_batch + kTrainTile - 1) / kTrainTile;
    if (hipMalloc(&S.feat, (size_t)n * 4 * sizeof(float)) != hipSuccess ||
        hipMalloc(&S.targ, (size_t)n * 8 * sizeof(float)) != hipSuccess ||
        hipMalloc(&S.gpart, (size_t)blocks * kMlpParams * sizeof(float)) != hipSuccess ||
        hipMalloc(&S.lpart, (size_t)blocks * sizeof(double)) != hipSuccess ||
        hipMalloc(&S.loss, sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KRT_E_NOMEM, "cannot allocate training scratch");
    }
    return KRT_OK;
}

// Loss over the whole prepared set (stored order), summed on the device.
krt_status mlp_set_loss(krt_ctx* ctx, MlpScratch& S, int64_t n, int64_t chunk, double* out_loss) {
    double total = 0.0;
    for (int64_t first = 0; first < n; first += chunk) {
        const int64_t cnt = std::min(chunk, n - first);
        const int blocks = mlp_pass(ctx, S.feat, S.targ, n, first, cnt, false, 0, 0, S.gpart, S.lpart);
        hipLaunchKernelGGL(mlp_loss_sum, dim3(1), dim3(64), 0, ctx->stream, S.lpart, blocks, S.loss);
        KRT_HIP(ctx, hipGetLastError());
        double h = 0.0;
        KRT_HIP(ctx, hipMemcpyAsync(&h, S.loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        total += h;
    }
    *out_loss = total / (8.0 * (double)n);
    return KRT_OK;
}

}  // namespace

extern "C" {

int krt_abi_version(void) { return KRT_ABI_VERSION; }

krt_status krt_check_camera(const krt_camera* cam, char* msg, size_t msg_len) {
    const std::string m = check_camera(cam);
    if (msg && msg_len > 0) {
        std::strncpy(msg, m.c_str(), msg_len - 1);
        msg[msg_len - 1] = '\0';
    }
    return m.empty() ? KRT_OK : KRT_E_INVAL;
}

krt_status krt_create(int device, krt_ctx** out) {
    if (!out) return KRT_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return KRT_E_INVAL;
    krt_ctx* ctx = new (std::nothrow) krt_ctx();
    if (!ctx) return KRT_E_NOMEM;
    ctx->device = device;
    krt_status st = KRT_OK;
    do {
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) { st = hip_fail(ctx, e, "hipSetDevice"); break; }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) { st = hip_fail(ctx, e, "hipGetDeviceProperties"); break; }
        ctx->cu_count = prop.multiProcessorCount;
        e = resolve_scratch(device);
        if (e != hipSuccess) { st = hip_fail(ctx, e, "hipGetSymbolAddress(scratch)"); break; }
        if (hipMalloc(&ctx->work, kWorkWords * sizeof(unsigned)) != hipSuccess ||
            hipMalloc(&ctx->red_partial, (kRedBlocks * 9 + 16) * sizeof(double)) != hipSuccess ||
            hipMalloc(&ctx->btab, (size_t)kBesPanels * 2 * kBesCoef * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&ctx->host_buf, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipEventCreate(&ctx->ev[0]) != hipSuccess || hipEventCreate(&ctx->ev[1]) != hipSuccess ||
            hipEventCreate(&ctx->ev[2]) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(ctx, KRT_E_NOMEM, "cannot allocate context buffers");
            break;
        }
        // Bessel-ratio table: node values, Chebyshev coefficients, then the
        // same polynomials in monomial form
        double* vals = nullptr;
        if (hipMalloc(&vals, (size_t)kBesPanels * kBesCoef * 2 * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(ctx, KRT_E_NOMEM, "cannot allocate table scratch");
            break;
        }
        const int nn = kBesPanels * kBesCoef;
        hipLaunchKernelGGL(bessel_table_nodes, dim3((nn + 127) / 128), dim3(128), 0, nullptr, vals);
        const int nc = kBesPanels * 2 * kBesCoef;
        hipLaunchKernelGGL(bessel_table_coefs, dim3((nc + 127) / 128), dim3(128), 0, nullptr, vals,
                           ctx->btab);
        hipLaunchKernelGGL(bessel_table_monomial, dim3((kBesPanels * 2 + 127) / 128), dim3(128), 0, nullptr,
                           ctx->btab);
        e = hipDeviceSynchronize();
        (void)hipFree(vals);
        if (e != hipSuccess) { st = hip_fail(ctx, e, "bessel table"); break; }
        e = hipGetLastError();
        if (e != hipSuccess) { st = hip_fail(ctx, e, "bessel table launch"); break; }
    } while (0);
    if (st != KRT_OK) {
        krt_destroy(ctx);
        return st;
    }
    *out = ctx;
    return KRT_OK;
}

krt_status krt_destroy(krt_ctx* ctx) {
    if (!ctx) return KRT_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->pool) (void)hipFree(ctx->pool);
    if (ctx->long_pool) (void)hipFree(ctx->long_pool);
    if (ctx->overflow_list) (void)hipFree(ctx->overflow_list);
    if (ctx->work) (void)hipFree(ctx->work);
    if (ctx->overflow_inst) (void)hipFree(ctx->overflow_inst);
    if (ctx->batch_dev) (void)hipFree(ctx->batch_dev);
    if (ctx->batch_host) (void)hipHostFree(ctx->batch_host);
    if (ctx->chunk_pool) (void)hipFree(ctx->chunk_pool);
    if (ctx->chunk_flags) (void)hipFree(ctx->chunk_flags);
    if (ctx->red_partial) (void)hipFree(ctx->red_partial);
    if (ctx->btab) (void)hipFree(ctx->btab);
    if (ctx->syntab) (void)hipFree(ctx->syntab);
    if (ctx->tile_order) (void)hipFree(ctx->tile_order);
    if (ctx->probe_dev) (void)hipFree(ctx->probe_dev);
    if (ctx->snap_copy) (void)hipFree(ctx->snap_copy);
    if (ctx->x2tab) (void)hipFree(ctx->x2tab);
    if (ctx->mlp_P) (void)hipFree(ctx->mlp_P);
    if (ctx->mlp_m) (void)hipFree(ctx->mlp_m);
    if (ctx->mlp_v) (void)hipFree(ctx->mlp_v);
    if (ctx->mlp_norm) (void)hipFree(ctx->mlp_norm);
    if (ctx->mlp_packed) (void)hipFree(ctx->mlp_packed);
    if (ctx->host_buf) (void)hipHostFree(ctx->host_buf);
    for (int k = 0; k < 3; ++k)
        if (ctx->ev[k]) (void)hipEventDestroy(ctx->ev[k]);
    delete ctx;
    return KRT_OK;
}

krt_status krt_set_stream(krt_ctx* ctx, void* hip_stream) {
    if (!ctx) return KRT_E_INVAL;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return KRT_OK;
}

krt_status krt_set_units(krt_ctx* ctx, const krt_units* u) {
    if (!ctx) return KRT_E_INVAL;
    const std::string m = krt_host::check_units(u);
    if (!m.empty()) return fail(ctx, KRT_E_INVAL, m);
    ctx->units = *u;
    ctx->units_set = true;
    return KRT_OK;
}

krt_status krt_set_model_adaf(krt_ctx* ctx, const krt_adaf* p) {
    if (!ctx) return KRT_E_INVAL;
    bool unsup = false;
    const std::string m = krt_host::check_adaf(p, &unsup);
    if (!m.empty()) return fail(ctx, unsup ? KRT_E_UNSUPPORTED : KRT_E_INVAL, m);
    ctx->adaf = *p;
    ctx->model = kModelAdaf;
    return KRT_OK;
}

krt_status krt_set_model_snapshot(krt_ctx* ctx, const krt_snapshot_desc* desc, const void* d_prims,
                                  int dtype) {
    if (!ctx) return KRT_E_INVAL;
    bool unsup = false;
    const std::string m = krt_host::check_snapshot(desc, d_prims, dtype, &unsup);
    if (!m.empty()) return fail(ctx, unsup ? KRT_E_UNSUPPORTED : KRT_E_INVAL, m);
    const krt_snapshot_desc& d = *desc;
    if (d.layout == 1) {
        // one transpose into the library's copy in the gather's layout (the
        // copy is read instead of d_prims from now on)
        const size_t ncell = (size_t)d.n1 * d.n2 * d.n3;
        const size_t esz = dtype == KRT_DTYPE_F64 ? sizeof(double) : sizeof(float);
        const size_t bytes = ncell * 8 * esz;
        KRT_HIP(ctx, hipSetDevice(ctx->device));
        if (ctx->snap_copy_bytes < bytes) {
            KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->snap_copy) KRT_HIP(ctx, hipFree(ctx->snap_copy));
            ctx->snap_copy = nullptr;
            ctx->snap_copy_bytes = 0;
            if (hipMalloc(&ctx->snap_copy, bytes) != hipSuccess) {
                (void)hipGetLastError();
                ctx->snap_copy = nullptr;
                return fail(ctx, KRT_E_NOMEM, "cannot allocate the snapshot copy for layout 1");
            }
            ctx->snap_copy_bytes = bytes;
        }
        const dim3 grid((unsigned)((ncell + 63) / 64));
        if (dtype == KRT_DTYPE_F64)
            hipLaunchKernelGGL(snapshot_to_cells<double>, grid, dim3(256), 0, ctx->stream,
                               static_cast<const double*>(d_prims), static_cast<double*>(ctx->snap_copy), ncell);
        else
            hipLaunchKernelGGL(snapshot_to_cells<float>, grid, dim3(256), 0, ctx->stream,
                               static_cast<const float*>(d_prims), static_cast<float*>(ctx->snap_copy), ncell);
        KRT_HIP(ctx, hipGetLastError());
        d_prims = ctx->snap_copy;
    }
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    if (!ctx->x2tab && hipMalloc(&ctx->x2tab, (kX2Tab + 1) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        ctx->x2tab = nullptr;
        return fail(ctx, KRT_E_NOMEM, "cannot allocate the MKS inversion table");
    }
    hipLaunchKernelGGL(mks_x2_table, dim3((kX2Tab + 128) / 128), dim3(128), 0, ctx->stream, d.hslope, ctx->x2tab);
    KRT_HIP(ctx, hipGetLastError());
    ctx->snap = d;
    ctx->snap_prims = dtype == KRT_DTYPE_F64 ? static_cast<const double*>(d_prims) : nullptr;
    ctx->snap_prims_f = dtype == KRT_DTYPE_F32 ? static_cast<const float*>(d_prims) : nullptr;
    ctx->model = kModelSnapshot;
    return KRT_OK;
}

krt_status krt_set_precision(krt_ctx* ctx, int precision) {
    if (!ctx) return KRT_E_INVAL;
    if (precision != KRT_PRECISION_FP64 && precision != KRT_PRECISION_FP32_TRANSFER)
        return fail(ctx, KRT_E_INVAL, "precision must be KRT_PRECISION_FP64 or KRT_PRECISION_FP32_TRANSFER");
    ctx->precision = precision;
    return KRT_OK;
}

}  // extern "C"

namespace {

// The plain tracer over the whole image, or (probe_np > 0) over the listed
// pixels, each traced by all 64 lanes of a wave (probe_host: host array).
krt_status trace_plain(krt_ctx* ctx, const krt_camera* cam, double* d_stokes, uint8_t* d_status,
                       int32_t* d_nsteps, krt_stats* out_stats, const int32_t* probe_host, int32_t probe_np) {
    krt_status st = check_ready(ctx, cam);
    if (st != KRT_OK) return st;
    if (!d_stokes) return fail(ctx, KRT_E_INVAL, "d_stokes is NULL");
    if (probe_np > 0) {
        const int64_t np = (int64_t)cam->nx * cam->ny;
        for (int32_t k = 0; k < probe_np; ++k)
            if (probe_host[k] < 0 || probe_host[k] >= np) return fail(ctx, KRT_E_INVAL, "probe pixel out of the image");
        if (ctx->electrons != KRT_ELECTRONS_THERMAL)
            return fail(ctx, KRT_E_UNSUPPORTED, "the probe traces thermal electrons only");
    }
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    const size_t npix = probe_np > 0 ? (size_t)probe_np * 64 : (size_t)cam->nx * cam->ny;
    const int el = ctx->electrons;
    const bool f32 = el == KRT_ELECTRONS_THERMAL && ctx->precision == KRT_PRECISION_FP32_TRANSFER;
    if (el == KRT_ELECTRONS_KAPPA_SURROGATE && !ctx->mlp_ready)
        return fail(ctx, KRT_E_STATE, "kappa surrogate selected but no surrogate parameters set");
    if (el != KRT_ELECTRONS_THERMAL && (st = ensure_syntab(ctx)) != KRT_OK) return st;
    if (el == KRT_ELECTRONS_KAPPA_SURROGATE) st = ensure_pool<kModeKapMlp>(ctx);
    else if (el == KRT_ELECTRONS_KAPPA_EXACT) st = ensure_pool<kModeKapExact>(ctx);
    else st = f32 ? ensure_pool<kModeF32>(ctx) : ensure_pool<kModeF64>(ctx);
    if (st != KRT_OK) return st;
    if ((st = ensure_chunks(ctx)) != KRT_OK) return st;
    if ((st = ensure_long(ctx, cam->max_steps, npix)) != KRT_OK) return st;
    TraceArgs A = base_args(ctx, cam);
    if ((st = ensure_tile_order(ctx, A.tiles_x, A.nbatch / A.tiles_x, A.tile_w, &A.tile_order, &A.nsec)) != KRT_OK)
        return st;
    A.kappa = ctx->kappa;
    A.syntab = ctx->syntab;
    A.mlp = ctx->mlp_packed;
    A.pool = ctx->pool;
    A.cap = ctx->pool_cap;
    A.chunk_pool = ctx->chunk_pool;
    A.chunk_flags = ctx->chunk_flags;
    A.nchunks = ctx->nchunks;
    if (ctx->nchunks > 0)
        KRT_HIP(ctx, hipMemsetAsync(ctx->chunk_flags, 0, (size_t)ctx->nchunks * sizeof(unsigned), ctx->stream));
    A.long_pool = ctx->long_pool;
    A.long_slots = ctx->long_slots;
    A.overflow_list = ctx->overflow_list;
    A.stokes = d_stokes;
    A.status = d_status;
    A.nsteps = d_nsteps;
    if (probe_np > 0) {
        if (ctx->probe_cap < (size_t)probe_np) {
            KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->probe_dev) KRT_HIP(ctx, hipFree(ctx->probe_dev));
            ctx->probe_dev = nullptr;
            ctx->probe_cap = 0;
            if (hipMalloc(&ctx->probe_dev, (size_t)probe_np * sizeof(int32_t)) != hipSuccess) {
                ctx->probe_dev = nullptr;
                (void)hipGetLastError();
                return fail(ctx, KRT_E_NOMEM, "cannot allocate the probe list");
            }
            ctx->probe_cap = (size_t)probe_np;
        }
        KRT_HIP(ctx, hipMemcpyAsync(ctx->probe_dev, probe_host, (size_t)probe_np * sizeof(int32_t),
                                    hipMemcpyHostToDevice, ctx->stream));
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        A.probe_pix = ctx->probe_dev;
        A.probe_np = probe_np;
        A.nbatch = probe_np;
        A.tile_order = nullptr;
        A.nsec = 1;
        A.status = nullptr;
        A.nsteps = nullptr;
    }
    KRT_HIP(ctx, hipMemsetAsync(ctx->work, 0, kWorkWords * sizeof(unsigned), ctx->stream));
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
    const dim3 grid(ctx->launch_blocks), lgrid(ctx->long_slots / 64);
    if (el == KRT_ELECTRONS_KAPPA_SURROGATE)
        hipLaunchKernelGGL(trace_waves<kModeKapMlp>, grid, dim3(256), 0, ctx->stream, A);
    else if (el == KRT_ELECTRONS_KAPPA_EXACT)
        hipLaunchKernelGGL(trace_waves<kModeKapExact>, grid, dim3(256), 0, ctx->stream, A);
    else if (f32)
        hipLaunchKernelGGL(trace_waves<kModeF32>, grid, dim3(256), 0, ctx->stream, A);
    else
        hipLaunchKernelGGL(trace_waves<kModeF64>, grid, dim3(256), 0, ctx->stream, A);
    KRT_HIP(ctx, hipGetLastError());
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
    if (probe_np > 0) {
        // no long-ray pass: a probe ray that outgrew the store is an error
        krt_stats s{};
        krt_stats* sp = out_stats ? out_stats : &s;
        KRT_HIP(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
        if ((st = fill_stats(ctx, (int64_t)npix, sp)) != KRT_OK) return st;
        if (sp->long_rays > 0) return fail(ctx, KRT_E_NOMEM, "a probe ray outgrew the path store");
        return KRT_OK;
    }
    // long rays of either kappa mode use the exact integrator
    if (el != KRT_ELECTRONS_THERMAL)
        hipLaunchKernelGGL(trace_long<kModeKapExact>, lgrid, dim3(64), 0, ctx->stream, A);
    else if (f32)
        hipLaunchKernelGGL(trace_long<kModeF32>, lgrid, dim3(64), 0, ctx->stream, A);
    else
        hipLaunchKernelGGL(trace_long<kModeF64>, lgrid, dim3(64), 0, ctx->stream, A);
    KRT_HIP(ctx, hipGetLastError());
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
    if (out_stats) return fill_stats(ctx, (int64_t)cam->nx * cam->ny, out_stats);
    return KRT_OK;
}

}  // namespace

extern "C" {

krt_status krt_trace_steps(krt_ctx* ctx, const krt_camera* cam, double* d_stokes, uint8_t* d_status,
                           int32_t* d_nsteps, krt_stats* out_stats) {
    return trace_plain(ctx, cam, d_stokes, d_status, d_nsteps, out_stats, nullptr, 0);
}

krt_status krt_trace(krt_ctx* ctx, const krt_camera* cam, double* d_stokes, uint8_t* d_status,
                     krt_stats* out_stats) {
    return trace_plain(ctx, cam, d_stokes, d_status, nullptr, out_stats, nullptr, 0);
}

krt_status krt_trace_probe(krt_ctx* ctx, const krt_camera* cam, const int32_t* pixels, int32_t npix,
                           double* d_stokes, krt_stats* out_stats) {
    if (!ctx) return KRT_E_INVAL;
    if (!pixels || npix < 1) return fail(ctx, KRT_E_INVAL, "empty probe pixel list");
    return trace_plain(ctx, cam, d_stokes, nullptr, nullptr, out_stats, pixels, npix);
}

krt_status krt_set_launch_config(krt_ctx* ctx, const krt_launch_config* cfg) {
    if (!ctx) return KRT_E_INVAL;
    const std::string m = krt_host::check_launch_config(cfg);
    if (!m.empty()) return fail(ctx, KRT_E_INVAL, m);
    ctx->cfg = *cfg;
    return KRT_OK;
}

krt_status krt_get_launch_config(const krt_ctx* ctx, krt_launch_config* out) {
    if (!ctx || !out) return KRT_E_INVAL;
    *out = ctx->cfg;
    return KRT_OK;
}

krt_status krt_trace_batch(krt_ctx* ctx, const krt_camera* groups, int32_t ngroups, const krt_instance* inst,
                           int32_t ninst, krt_stats* out_stats) {
    if (!ctx) return KRT_E_INVAL;
    if (!groups || ngroups < 1 || ngroups > 4096) return fail(ctx, KRT_E_INVAL, "need 1..4096 groups");
    if (!inst || ninst < 1 || ninst > (1 << 20)) return fail(ctx, KRT_E_INVAL, "need 1..2^20 instances");
    krt_status st = check_ready(ctx, &groups[0]);
    if (st != KRT_OK) return st;
    for (int g = 0; g < ngroups; ++g) {
        const std::string m = check_camera(&groups[g]);
        if (!m.empty()) return fail(ctx, KRT_E_INVAL, "group " + std::to_string(g) + ": " + m);
        if (groups[g].a != groups[0].a || groups[g].mass_factor != groups[0].mass_factor)
            return fail(ctx, KRT_E_INVAL, "all groups must share the spin and mass factor");
    }
    std::vector<int> count(ngroups, 0);
    int64_t rays = 0;
    for (int q = 0; q < ninst; ++q) {
        const krt_instance& I = inst[q];
        if (I.struct_size != sizeof(krt_instance)) return fail(ctx, KRT_E_INVAL, "instance struct_size mismatch");
        if (I.group < 0 || I.group >= ngroups) return fail(ctx, KRT_E_INVAL, "instance group out of range");
        if (!std::isfinite(I.freq_hz) || !(I.freq_hz > 0.0)) return fail(ctx, KRT_E_INVAL, "instance freq_hz must be > 0");
        if (!std::isfinite(I.M_unit_g) || I.M_unit_g < 0.0 || !std::isfinite(I.R_high) || I.R_high < 0.0)
            return fail(ctx, KRT_E_INVAL, "instance M_unit_g and R_high must be finite and >= 0");
        if (ctx->model != kModelSnapshot && (I.M_unit_g != 0.0 || I.R_high != 0.0))
            return fail(ctx, KRT_E_INVAL, "M_unit_g and R_high apply to the snapshot model only (use 0)");
        if (!I.d_stokes) return fail(ctx, KRT_E_INVAL, "instance d_stokes is NULL");
        ++count[I.group];
        rays += (int64_t)groups[I.group].nx * groups[I.group].ny;
    }
    if (rays > (int64_t)INT32_MAX) return fail(ctx, KRT_E_INVAL, "more than 2^31 instance pixels");
    // queue order of the groups: most instances first (their tiles cost most)
    std::vector<int> gorder(ngroups);
    for (int g = 0; g < ngroups; ++g) gorder[g] = g;
    if (ctx->cfg.order >= 1)
        std::stable_sort(gorder.begin(), gorder.end(), [&](int x, int y) { return count[x] > count[y]; });
    std::vector<int> gpos(ngroups);
    for (int k = 0; k < ngroups; ++k) gpos[gorder[k]] = k;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    const bool f32 = ctx->precision == KRT_PRECISION_FP32_TRANSFER;
    if ((st = f32 ? ensure_pool<kModeF32>(ctx, true) : ensure_pool<kModeF64>(ctx, true)) != KRT_OK) return st;
    if ((st = ensure_chunks(ctx)) != KRT_OK) return st;
    int max_steps = 1;
    for (int g = 0; g < ngroups; ++g) max_steps = std::max(max_steps, (int)groups[g].max_steps);
    if ((st = ensure_long(ctx, max_steps, (size_t)rays)) != KRT_OK) return st;

    // descriptors: groups in queue order, instances sorted by group
    const int tw = ctx->cfg.tile_w, thh = 64 / tw;
    std::vector<GroupDev> G(ngroups);
    int items = 0;
    std::vector<int> ibegin(ngroups + 1, 0);
    for (int k = 0; k < ngroups; ++k) ibegin[k + 1] = ibegin[k] + count[gorder[k]];
    for (int k = 0; k < ngroups; ++k) {
        const krt_camera& c = groups[gorder[k]];
        GroupDev& d = G[k];
        std::memset(&d, 0, sizeof(d));
        d.cam = camera_desc(&c);
        d.eps = c.eps;
        d.r_stop = c.mass_factor == 0 ? 1e-6 : 1.05 * horizon(c.a, 1.0);
        d.max_steps = c.max_steps;
        d.tiles_x = (c.nx + tw - 1) / tw;
        d.item_begin = items;
        items += d.tiles_x * ((c.ny + thh - 1) / thh);
        d.item_end = items;
        d.inst_begin = ibegin[k];
        d.inst_end = ibegin[k + 1];
    }
    std::vector<InstDev> I(ninst);
    std::vector<int> fill(ngroups, 0);
    for (int q = 0; q < ninst; ++q) {
        const int k = gpos[inst[q].group];
        const int slotq = ibegin[k] + fill[k]++;
        krt_camera c = groups[inst[q].group];
        c.freq_hz = inst[q].freq_hz;
        TraceArgs T = base_args(ctx, &c);
        if (ctx->model == kModelSnapshot) {
            const double L = T.L_cm;
            if (inst[q].M_unit_g > 0.0) {
                T.snap.rho_unit = inst[q].M_unit_g / (L * L * L);
                T.snap.B_unit = kC * std::sqrt(4.0 * kPi * T.snap.rho_unit);
            }
            if (inst[q].R_high > 0.0) T.snap.Rhigh = inst[q].R_high;
            fill_f32(ctx, c.freq_hz, T);
        }
        InstDev& d = I[slotq];
        std::memset(&d, 0, sizeof(d));
        d.freq = c.freq_hz;
        d.fac0 = T.fac0;
        d.rho_unit = T.snap.rho_unit;
        d.B_unit = T.snap.B_unit;
        d.Rhigh = T.snap.Rhigh;
        d.f32 = T.f32;
        d.stokes = inst[q].d_stokes;
        d.status = inst[q].d_status;
        d.group = k;
    }
    const size_t gbytes = (size_t)ngroups * sizeof(GroupDev), ibytes = (size_t)ninst * sizeof(InstDev);
    const size_t ioff = (gbytes + 255) / 256 * 256, need = ioff + ibytes;
    if (ctx->batch_host_bytes < need || ctx->batch_dev_bytes < need) {
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->batch_host) KRT_HIP(ctx, hipHostFree(ctx->batch_host));
        if (ctx->batch_dev) KRT_HIP(ctx, hipFree(ctx->batch_dev));
        ctx->batch_host = ctx->batch_dev = nullptr;
        ctx->batch_host_bytes = ctx->batch_dev_bytes = 0;
        if (hipHostMalloc(&ctx->batch_host, need) != hipSuccess || hipMalloc(&ctx->batch_dev, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, KRT_E_NOMEM, "cannot allocate the batch descriptors");
        }
        ctx->batch_host_bytes = ctx->batch_dev_bytes = need;
    } else {
        // the staging buffer may still feed an earlier batch's copy
        KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    char* hb = static_cast<char*>(ctx->batch_host);
    std::memcpy(hb, G.data(), gbytes);
    std::memcpy(hb + ioff, I.data(), ibytes);
    KRT_HIP(ctx, hipMemcpyAsync(ctx->batch_dev, ctx->batch_host, need, hipMemcpyHostToDevice, ctx->stream));

    TraceArgs A = base_args(ctx, &groups[gorder[0]]);
    A.groups = reinterpret_cast<const GroupDev*>(ctx->batch_dev);
    A.inst = reinterpret_cast<const InstDev*>(static_cast<char*>(ctx->batch_dev) + ioff);
    A.ngroups = ngroups;
    A.nbatch = items;
    A.max_steps = max_steps;
    A.pool = ctx->pool;
    A.cap = ctx->pool_cap;
    A.chunk_pool = ctx->chunk_pool;
    A.chunk_flags = ctx->chunk_flags;
    A.nchunks = ctx->nchunks;
    A.long_pool = ctx->long_pool;
    A.long_slots = ctx->long_slots;
    A.overflow_list = ctx->overflow_list;
    A.overflow_inst = ctx->overflow_inst;
    if (ctx->nchunks > 0)
        KRT_HIP(ctx, hipMemsetAsync(ctx->chunk_flags, 0, (size_t)ctx->nchunks * sizeof(unsigned), ctx->stream));
    KRT_HIP(ctx, hipMemsetAsync(ctx->work, 0, kWorkWords * sizeof(unsigned), ctx->stream));
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
    if (f32)
        hipLaunchKernelGGL(trace_batch<kModeF32>, dim3(ctx->launch_blocks), dim3(256), 0, ctx->stream, A);
    else
        hipLaunchKernelGGL(trace_batch<kModeF64>, dim3(ctx->launch_blocks), dim3(256), 0, ctx->stream, A);
    KRT_HIP(ctx, hipGetLastError());
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
    if (f32)
        hipLaunchKernelGGL(trace_long<kModeF32>, dim3(ctx->long_slots / 64), dim3(64), 0, ctx->stream, A);
    else
        hipLaunchKernelGGL(trace_long<kModeF64>, dim3(ctx->long_slots / 64), dim3(64), 0, ctx->stream, A);
    KRT_HIP(ctx, hipGetLastError());
    if (out_stats) KRT_HIP(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
    if (out_stats) return fill_stats(ctx, rays, out_stats);
    return KRT_OK;
}

krt_status krt_autotune(krt_ctx* ctx, const krt_camera* groups, int32_t ngroups, const krt_instance* inst,
                        int32_t ninst, const char* cache_path, krt_launch_config* out_cfg) {
    if (!ctx) return KRT_E_INVAL;
    if (!groups || ngroups < 1 || !inst || ninst < 1) return fail(ctx, KRT_E_INVAL, "empty batch");
    // cache key: device, precision, model and the batch's shape
    hipDeviceProp_t prop;
    KRT_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    std::string key = std::string(prop.gcnArchName) + "|" + std::to_string(ctx->cu_count) + "|p" +
                      std::to_string(ctx->precision) + "|m" + std::to_string(ctx->model);
    std::vector<int> per(ngroups, 0);
    for (int q = 0; q < ninst; ++q)
        if (inst[q].group >= 0 && inst[q].group < ngroups) ++per[inst[q].group];
    for (int g = 0; g < ngroups; ++g)
        key += "|" + std::to_string(groups[g].nx) + "x" + std::to_string(groups[g].ny) + "i" + std::to_string(per[g]);
    unsigned long long h = 1469598103934665603ULL;  // FNV-1a
    for (unsigned char ch : key) {
        h ^= ch;
        h *= 1099511628211ULL;
    }
    char hkey[32];
    std::snprintf(hkey, sizeof(hkey), "%016llx", h);
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char k[64];
            krt_launch_config c{sizeof(krt_launch_config), 8, 0, 0, 1};
            double ms = 0.0;
            bool found = false;
            while (std::fscanf(f, "%63s %d %d %d %d %lf", k, &c.tile_w, &c.blocks_per_cu, &c.path_cap, &c.order, &ms) == 6)
                if (std::strcmp(k, hkey) == 0) found = true, ctx->cfg = c;
            std::fclose(f);
            if (found) {
                if (out_cfg) *out_cfg = ctx->cfg;
                return KRT_OK;
            }
        }
    }
    // reduced batch: the first instance of every group
    std::vector<krt_instance> red;
    std::vector<char> seen(ngroups, 0);
    for (int q = 0; q < ninst; ++q) {
        const int g = inst[q].group;
        if (g >= 0 && g < ngroups && !seen[g]) {
            seen[g] = 1;
            red.push_back(inst[q]);
        }
    }
    const krt_launch_config saved = ctx->cfg;
    krt_launch_config best = saved;
    double best_ms = 1e300;
    const int tws[] = {8, 16, 32}, bpcs[] = {1, 2}, caps[] = {4096, 8192};
    for (int tw : tws)
        for (int bpc : bpcs)
            for (int cap : caps) {
                krt_launch_config c{sizeof(krt_launch_config), tw, bpc, cap, 1};
                ctx->cfg = c;
                krt_stats stt;
                stt.struct_size = sizeof(krt_stats);
                const krt_status e = krt_trace_batch(ctx, groups, ngroups, red.data(), (int32_t)red.size(), &stt);
                if (e != KRT_OK) {
                    ctx->cfg = saved;
                    return e;
                }
                const double ms = stt.kernel_ms[0] + stt.kernel_ms[1];
                if (ms < best_ms) best_ms = ms, best = c;
            }
    ctx->cfg = best;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s %d %d %d %d %.3f\n", hkey, best.tile_w, best.blocks_per_cu, best.path_cap, best.order,
                         best_ms);
            std::fclose(f);
        }
    }
    if (out_cfg) *out_cfg = best;
    return KRT_OK;
}

krt_status krt_geodesic_only(krt_ctx* ctx, const krt_camera* cam, double* d_end_state,
                             int32_t* d_nsteps, uint8_t* d_status, double* d_invariant_drift) {
    if (!ctx) return KRT_E_INVAL;
    const std::string m = check_camera(cam);
    if (!m.empty()) return fail(ctx, KRT_E_INVAL, m);
    if (!d_end_state) return fail(ctx, KRT_E_INVAL, "d_end_state is NULL");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    TraceArgs A = base_args(ctx, cam);
    A.end_state = d_end_state;
    A.nsteps = d_nsteps;
    A.status = d_status;
    A.drift = d_invariant_drift;
    int per_cu = 0;
    KRT_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_waves<kModeGeo>, 256, 0));
    const int blocks = (per_cu < 1 ? 1 : per_cu) * ctx->cu_count;
    KRT_HIP(ctx, hipMemsetAsync(ctx->work, 0, kWorkWords * sizeof(unsigned), ctx->stream));
    hipLaunchKernelGGL(trace_waves<kModeGeo>, dim3(blocks), dim3(256), 0, ctx->stream, A);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

}  // extern "C"

namespace {

// The image reduction with its block partials and results in `partial`
// (kScratchDoubles doubles: the context's buffer or the static scratch).
krt_status reduce_into(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam, double out_flux_jy[4],
                       double* out_imax, double* partial) {
    const size_t np = (size_t)cam->nx * cam->ny;
    const double L = kG * ctx->units.M_bh_g / (kC * kC);
    const double D = ctx->units.dist_cm;
    const double dOm = (cam->fov_x * L / (cam->nx * D)) * (cam->fov_y * L / (cam->ny * D));
    int nb = (int)((np + 255) / 256);
    if (nb > kRedBlocks) nb = kRedBlocks;
    // every partial read below is written first: nothing needs clearing
    hipLaunchKernelGGL(reduce_partial, dim3(nb), dim3(256), 0, ctx->stream, d_stokes, np, partial);
    KRT_HIP(ctx, hipGetLastError());
    double* out = partial + (size_t)kRedBlocks * 9;  // 16 doubles after the partials
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(1), 0, ctx->stream, partial, nb, 1e23 * dOm, out);
    KRT_HIP(ctx, hipGetLastError());
    KRT_HIP(ctx, hipMemcpyAsync(ctx->host_buf, out, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 4; ++k) out_flux_jy[k] = ctx->host_buf[k];
    *out_imax = ctx->host_buf[4];
    return KRT_OK;
}

krt_status reduce_checks(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam, double out_flux_jy[4],
                         double* out_imax) {
    const std::string m = check_camera(cam);
    if (!m.empty()) return fail(ctx, KRT_E_INVAL, m);
    if (!d_stokes || !out_flux_jy || !out_imax) return fail(ctx, KRT_E_INVAL, "NULL argument");
    if (!ctx->units_set) return fail(ctx, KRT_E_STATE, "units not set");
    return KRT_OK;
}

}  // namespace

extern "C" {

krt_status krt_reduce(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam, double out_flux_jy[4],
                      double* out_imax) {
    if (!ctx) return KRT_E_INVAL;
    krt_status st = reduce_checks(ctx, d_stokes, cam, out_flux_jy, out_imax);
    if (st != KRT_OK) return st;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    return reduce_into(ctx, d_stokes, cam, out_flux_jy, out_imax, ctx->red_partial);
}

krt_status krt_reduce_noalloc(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam,
                              double out_flux_jy[4], double* out_imax) {
    if (!ctx) return KRT_E_INVAL;
    krt_status st = reduce_checks(ctx, d_stokes, cam, out_flux_jy, out_imax);
    if (st != KRT_OK) return st;
    if (ctx->device >= kMaxDevices) return fail(ctx, KRT_E_UNSUPPORTED, "device index above the scratch table");
    static_assert((size_t)kRedBlocks * 9 + 5 <= kScratchDoubles, "scratch holds the partials and the results");
    double* partial = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        partial = g_scratch_dev[ctx->device];
    }
    if (!partial) return fail(ctx, KRT_E_STATE, "static scratch of this device not resolved");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    return reduce_into(ctx, d_stokes, cam, out_flux_jy, out_imax, partial);
}

const char* krt_last_error(const krt_ctx* ctx) {
    if (!ctx) return "NULL context";
    return ctx->err.c_str();
}

krt_status krt_plasma_eval(krt_ctx* ctx, int64_t n, double a, int32_t mass_factor, const double* d_X,
                           double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_X || !d_out))) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (!(std::fabs(a) < 1.0) || (mass_factor != 0 && mass_factor != 1))
        return fail(ctx, KRT_E_INVAL, "bad spin or mass factor");
    if (ctx->model < 0) return fail(ctx, KRT_E_STATE, "no plasma model set");
    if (ctx->model == kModelSnapshot && !ctx->units_set) return fail(ctx, KRT_E_STATE, "units not set");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    krt_camera cam{};
    cam.a = a;
    cam.mass_factor = mass_factor;
    TraceArgs A = base_args(ctx, &cam);
    A.adaf.risco = isco(a);
    hipLaunchKernelGGL(hook_plasma, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream, A, n, a,
                       (double)mass_factor, d_X, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

krt_status krt_coeffs(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(hook_coeffs, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream, ctx->btab, n,
                       d_in, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

krt_status krt_bessel_ratios(krt_ctx* ctx, int64_t n, const double* d_x, double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_x || !d_out))) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(hook_bessel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream, ctx->btab, n,
                       d_x, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

krt_status krt_mueller_step(krt_ctx* ctx, int64_t n, const double* d_coef, const double* d_S, double w,
                            double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_coef || !d_S || !d_out)) || !std::isfinite(w) || w < 0.0)
        return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(hook_mueller, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream, n, d_coef,
                       d_S, w, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}


krt_status krt_set_electrons(krt_ctx* ctx, int kind, double kappa) {
    if (!ctx) return KRT_E_INVAL;
    if (kind != KRT_ELECTRONS_THERMAL && kind != KRT_ELECTRONS_KAPPA_EXACT && kind != KRT_ELECTRONS_KAPPA_SURROGATE)
        return fail(ctx, KRT_E_INVAL, "unknown electron distribution");
    if (kind != KRT_ELECTRONS_THERMAL && !(std::isfinite(kappa) && kappa > 2.0))
        return fail(ctx, KRT_E_INVAL, "kappa must be finite and > 2");
    ctx->electrons = kind;
    if (kind != KRT_ELECTRONS_THERMAL) ctx->kappa = kappa;
    return KRT_OK;
}

krt_status krt_kappa_integrals(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    krt_status st = ensure_syntab(ctx);
    if (st != KRT_OK) return st;
    hipLaunchKernelGGL(hook_kappa_integrals, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, ctx->stream,
                       ctx->syntab, n, d_in, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

krt_status krt_probe_fma(krt_ctx* ctx, int32_t blocks, int32_t iters, int32_t chains, double* out_ms) {
    if (!ctx) return KRT_E_INVAL;
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 24) || !out_ms ||
        (chains != 1 && chains != 2 && chains != 4 && chains != 8))
        return fail(ctx, KRT_E_INVAL, "probe needs blocks 1..2^20, iters 1..2^24, chains 1, 2, 4 or 8");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    double* d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, KRT_E_NOMEM, "probe buffer");
    }
    // x < 1 and y small: every chain converges to y / (1 - x), finite
    const double x = 0.999999, y = 1e-6;
    const hipError_t re = hipEventRecord(ctx->ev[0], ctx->stream);
    if (re != hipSuccess) {
        (void)hipFree(d);
        KRT_HIP(ctx, re);
    }
    switch (chains) {
        case 1: hipLaunchKernelGGL(fma_probe<1>, dim3(blocks), dim3(256), 0, ctx->stream, d, iters, x, y); break;
        case 2: hipLaunchKernelGGL(fma_probe<2>, dim3(blocks), dim3(256), 0, ctx->stream, d, iters, x, y); break;
        case 4: hipLaunchKernelGGL(fma_probe<4>, dim3(blocks), dim3(256), 0, ctx->stream, d, iters, x, y); break;
        default: hipLaunchKernelGGL(fma_probe<8>, dim3(blocks), dim3(256), 0, ctx->stream, d, iters, x, y); break;
    }
    const hipError_t le = hipGetLastError();
    const hipError_t re1 = hipEventRecord(ctx->ev[1], ctx->stream);
    const hipError_t se = re1 == hipSuccess ? hipEventSynchronize(ctx->ev[1]) : re1;
    float ms = 0.0f;
    const hipError_t te = (le == hipSuccess && se == hipSuccess) ? hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1])
                                                                  : hipSuccess;
    (void)hipFree(d);
    KRT_HIP(ctx, le);
    KRT_HIP(ctx, se);
    KRT_HIP(ctx, te);
    *out_ms = ms;
    return KRT_OK;
}

krt_status krt_mueller_general(krt_ctx* ctx, int64_t n, const double* d_coef, const double* d_S, double w,
                               double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_coef || !d_S || !d_out)) || !std::isfinite(w) || w < 0.0)
        return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(hook_mueller_general, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, ctx->stream, n,
                       d_coef, d_S, w, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

krt_status krt_mlp_set_params(krt_ctx* ctx, const float* params, const double* norm) {
    if (!ctx) return KRT_E_INVAL;
    if (!params || !norm) return fail(ctx, KRT_E_INVAL, "params and norm are required");
    for (int k = 0; k < kMlpParams; ++k)
        if (!std::isfinite(params[k])) return fail(ctx, KRT_E_INVAL, "non-finite parameter");
    for (int k = 0; k < kNormLen; ++k)
        if (!std::isfinite(norm[k]) || (k >= 8 && k < 16 && !(norm[k] > 0.0)))
            return fail(ctx, KRT_E_INVAL, "norm must be finite with positive sd");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    krt_status st = ensure_mlp(ctx);
    if (st != KRT_OK) return st;
    KRT_HIP(ctx, hipMemcpyAsync(ctx->mlp_P, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    KRT_HIP(ctx, hipMemcpyAsync(ctx->mlp_norm, norm, kNormLen * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    KRT_HIP(ctx, hipMemsetAsync(ctx->mlp_m, 0, kMlpParams * sizeof(float), ctx->stream));
    KRT_HIP(ctx, hipMemsetAsync(ctx->mlp_v, 0, kMlpParams * sizeof(float), ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return mlp_repack(ctx);
}

krt_status krt_mlp_get_params(krt_ctx* ctx, float* params, double* norm) {
    if (!ctx) return KRT_E_INVAL;
    if (!params || !norm) return fail(ctx, KRT_E_INVAL, "params and norm are required");
    if (!ctx->mlp_ready) return fail(ctx, KRT_E_STATE, "no surrogate parameters set");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    KRT_HIP(ctx, hipMemcpyAsync(params, ctx->mlp_P, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    KRT_HIP(ctx, hipMemcpyAsync(norm, ctx->mlp_norm, kNormLen * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KRT_OK;
}

krt_status krt_mlp_init(krt_ctx* ctx, uint64_t seed) {
    if (!ctx) return KRT_E_INVAL;
    std::vector<float> P(kMlpParams, 0.0f);
    uint64_t s = seed;
    auto fill = [&](int off, int rows, int fan_in) {
        const double b = std::sqrt(3.0 / fan_in) * 1.4142135623730951;
        for (int k = 0; k < rows * fan_in; ++k) {
            const double u = (double)(splitmix_next(s) >> 11) * 0x1.0p-53;
            P[off + k] = (float)((2.0 * u - 1.0) * b);
        }
    };
    fill(kOffW1, kMlpH, kMlpIn);
    fill(kOffW2, kMlpH, kMlpH);
    fill(kOffW3, kMlpH, kMlpH);
    fill(kOffW4, kMlpOut, kMlpH);
    std::vector<double> norm(kNormLen, 0.0);
    for (int k = 8; k < 16; ++k) norm[k] = 1.0;
    return krt_mlp_set_params(ctx, P.data(), norm.data());
}

krt_status krt_mlp_grad(krt_ctx* ctx, int64_t n, const double* d_in, const double* d_integ, float* d_grad,
                        double* out_loss) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 1 || n > (int64_t)1 << 24 || !d_in || !d_integ || !d_grad)
        return fail(ctx, KRT_E_INVAL, "bad arguments (1 <= n <= 2^24)");
    if (!ctx->mlp_ready) return fail(ctx, KRT_E_STATE, "no surrogate parameters set");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    MlpScratch S;
    krt_status st = mlp_scratch(ctx, S, n, n);
    if (st != KRT_OK) return st;
    hipLaunchKernelGGL(mlp_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n, d_in, d_integ,
                       ctx->mlp_norm, S.feat, S.targ);
    const int blocks = mlp_pass(ctx, S.feat, S.targ, n, 0, n, false, 0, 0, S.gpart, S.lpart);
    MlpStepArgs G{};
    G.gpart = S.gpart;
    G.nparts = blocks;
    G.grad = d_grad;
    hipLaunchKernelGGL(mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, G);
    hipLaunchKernelGGL(mlp_loss_sum, dim3(1), dim3(64), 0, ctx->stream, S.lpart, blocks, S.loss);
    KRT_HIP(ctx, hipGetLastError());
    double h = 0.0;
    KRT_HIP(ctx, hipMemcpyAsync(&h, S.loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    KRT_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (out_loss) *out_loss = h / (8.0 * (double)n);
    return KRT_OK;
}

krt_status krt_mlp_train(krt_ctx* ctx, int64_t n, const double* d_in, const double* d_integ,
                         const krt_train_config* cfg, double* out_loss) {
    if (!ctx) return KRT_E_INVAL;
    if (!cfg || cfg->struct_size != sizeof(krt_train_config)) return fail(ctx, KRT_E_INVAL, "bad train config");
    if (n < 32 || n > (int64_t)1 << 24 || !d_in || !d_integ) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (cfg->epochs < 1 || cfg->batch < 32 || cfg->batch % kTrainTile != 0 || cfg->batch > (1 << 20) ||
        !(cfg->lr_max > 0.0) || !(cfg->lr_min >= 0.0) || !(cfg->warmup_frac >= 0.0 && cfg->warmup_frac < 1.0))
        return fail(ctx, KRT_E_INVAL, "bad train config values");
    if (!ctx->mlp_ready) return fail(ctx, KRT_E_STATE, "no surrogate parameters set (krt_mlp_init)");
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t batch = std::min<int64_t>(cfg->batch, n);
    MlpScratch S;
    krt_status st = mlp_scratch(ctx, S, n, batch);
    if (st != KRT_OK) return st;
    if (cfg->set_norm) {
        st = mlp_fit_baseline(ctx, n, d_in, d_integ);
        if (st != KRT_OK) return st;
    }
    hipLaunchKernelGGL(mlp_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n, d_in, d_integ,
                       ctx->mlp_norm, S.feat, S.targ);
    KRT_HIP(ctx, hipMemsetAsync(ctx->mlp_m, 0, kMlpParams * sizeof(float), ctx->stream));
    KRT_HIP(ctx, hipMemsetAsync(ctx->mlp_v, 0, kMlpParams * sizeof(float), ctx->stream));
    const bool pow2 = (n & (n - 1)) == 0;
    const int64_t steps_per_epoch = (n + batch - 1) / batch;
    const int64_t total = steps_per_epoch * cfg->epochs;
    const int64_t warm = (int64_t)(cfg->warmup_frac * (double)total);
    uint64_t rs = cfg->seed;
    int64_t step = 0;
    const double b1 = 0.9, b2 = 0.999;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        const uint64_t a = pow2 ? (splitmix_next(rs) | 1ull) : 1ull;
        const uint64_t c = pow2 ? splitmix_next(rs) : 0ull;
        for (int64_t first = 0; first < n; first += batch) {
            const int64_t cnt = std::min(batch, n - first);
            const int blocks = mlp_pass(ctx, S.feat, S.targ, n, first, cnt, pow2, a, c, S.gpart, S.lpart);
            ++step;
            double lr;
            if (step <= warm) lr = cfg->lr_max * (double)step / (double)warm;
            else {
                const double f = (double)(step - warm) / (double)std::max<int64_t>(1, total - warm);
                lr = cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) * (1.0 + std::cos(kPi * f));
            }
            MlpStepArgs G{};
            G.P = ctx->mlp_P;
            G.m = ctx->mlp_m;
            G.v = ctx->mlp_v;
            G.gpart = S.gpart;
            G.nparts = blocks;
            G.grad = nullptr;
            G.lr = (float)lr;
            G.beta1 = (float)b1;
            G.beta2 = (float)b2;
            G.eps = 1e-8f;
            G.bc1 = (float)(1.0 - std::pow(b1, (double)step));
            G.bc2 = (float)(1.0 - std::pow(b2, (double)step));
            hipLaunchKernelGGL(mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, ctx->stream, G);
        }
        KRT_HIP(ctx, hipGetLastError());
    }
    st = mlp_repack(ctx);
    if (st != KRT_OK) return st;
    double loss = 0.0;
    st = mlp_set_loss(ctx, S, n, batch, &loss);
    if (st != KRT_OK) return st;
    if (out_loss) *out_loss = loss;
    return KRT_OK;
}

krt_status krt_mlp_eval(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out) {
    if (!ctx) return KRT_E_INVAL;
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return fail(ctx, KRT_E_INVAL, "bad arguments");
    if (!ctx->mlp_ready) return fail(ctx, KRT_E_STATE, "no surrogate parameters set");
    if (n == 0) return KRT_OK;
    KRT_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(hook_mlp_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                       ctx->mlp_packed, n, d_in, d_out);
    KRT_HIP(ctx, hipGetLastError());
    return KRT_OK;
}

}  // extern "C"
