// C ABI (include/lbm.h) and host runtime: run handles, geometry and tile classification,
// device buffers through the allocator hook, step sequencing with HIP graphs, per-class
// timing, batched groups, autotuning and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

// A roctx range for the lifetime of the object when `on` (LBM_DEBUG_RANGES): rocprofv3
// --marker-trace records it, and outside a profiler the calls do nothing.
struct TraceRange {
    bool on;
    TraceRange(bool enable, const char *fmt, ...) : on(enable) {
        if (!on) return;
        char name[96];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(name, sizeof name, fmt, ap);
        va_end(ap);
        roctxRangePushA(name);
    }
    ~TraceRange() {
        if (on) roctxRangePop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

thread_local std::string g_err;

lbm_status fail(lbm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int storage) { return storage == ST_F64 ? 8 : storage == ST_F32 ? 4 : 2; }
size_t compute_size(int storage) { return storage == ST_F64 ? 8 : 4; }
long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

// Device buffers of one owner, through the caller's allocator hook or hipMalloc.  Every live
// buffer is kept with its size, so the owner can check that no two of them overlap (a hook that
// hands out aliasing memory would let one buffer's writes land in another's reads).
struct DeviceMem {
    const lbm_allocator *alloc = nullptr;
    std::vector<void *> ptrs;
    std::vector<size_t> sizes;
    void *get(size_t bytes) {
        void *p = nullptr;
        bytes = (size_t)round_up((long long)std::max<size_t>(bytes, 256), 256);
        if (alloc && alloc->alloc) p = alloc->alloc(bytes, alloc->ctx);
        else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
        if (p) { ptrs.push_back(p); sizes.push_back(bytes); }
        return p;
    }
    void put(void *p) {
        if (!p) return;
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            sizes.erase(sizes.begin() + (it - ptrs.begin()));
            ptrs.erase(it);
        }
        if (alloc && alloc->free) alloc->free(p, alloc->ctx);
        else (void)hipFree(p);
    }
    void release_all() {
        for (void *p : ptrs) {
            if (alloc && alloc->free) alloc->free(p, alloc->ctx);
            else (void)hipFree(p);
        }
        ptrs.clear();
        sizes.clear();
    }
    // true if two live buffers share a byte
    bool overlapping() const {
        std::vector<std::pair<uintptr_t, size_t>> r(ptrs.size());
        for (size_t k = 0; k < ptrs.size(); ++k) r[k] = {(uintptr_t)ptrs[k], sizes[k]};
        std::sort(r.begin(), r.end());
        for (size_t k = 1; k < r.size(); ++k)
            if (r[k].first < r[k - 1].first + r[k - 1].second) return true;
        return false;
    }
};

int tx_index(int tx) { return tx == 64 ? 0 : tx == 128 ? 1 : 2; }

// Side stream and events of the per-step fork/join: the bulk kernel runs on the main stream while
// the boundary chain (phase A, then the frame kernel) runs beside it on the side stream.  Both
// streams keep the default priority.
struct StepStreams {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, done = nullptr;
    bool ok = false;
    hipError_t create() {
        hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        ok = e == hipSuccess;
        return e;
    }
    void destroy() {
        if (side) (void)hipStreamDestroy(side);
        if (fork) (void)hipEventDestroy(fork);
        if (done) (void)hipEventDestroy(done);
        side = nullptr; fork = done = nullptr;
        ok = false;
    }
};

}  // namespace

struct lbm_run {
    lbm_desc desc{};
    lbm_allocator alloc_copy{};
    int pml[4] = {0, 0, 0, 0};
    int W = 0;
    double sigma_max = 0.0;
    int bc[4] = {BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC};
    unsigned pml_terms = 0;
    bool inited = false;
    RunDev hd{};
    RunDev *dd = nullptr;
    RunDev **dptr = nullptr;
    int *dprefix = nullptr;   // [NCLS][2] prefix arrays of the single-run launch set
    int nblocks[NCLS] = {0, 0, 0, 0};
    const LatticeInfo *lat = &LATTICE_D2Q37;   // velocity stencil
    const KernelSet *ks = &k37::kernels;       // its kernels
    double fbar[NQ_MAX];
    double *fbar_d = nullptr;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;     // stream in use (the group's while in a group)
    lbm_launch launch{64, 4, 32, 2, -1};
    int64_t steps = 0;
    DeviceMem mem;
    hipGraphExec_t graph = nullptr;
    int graph_G = 0;
    int graph_tx = 0;
    int graph_ov = 0;
    int graph_split = -1;
    bool graph_failed = false;
    int prof = 0;                     // 0 off, 1 classes in order, 2 bulk kernel in the normal schedule,
                                      // 3 as 2 on the first step of each batch only
    struct Ev { hipEvent_t a, b; int cls; };
    std::vector<Ev> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_n[3] = {0, 0, 0};
    lbm_group *group = nullptr;
    size_t footprint = 0;
    int *dflag = nullptr;             // lbm_check's flag, allocated with the run
    unsigned debug = 0;               // lbm_set_debug flags
    int64_t check_every = 0;          // lbm_set_check_interval: steps between checks in lbm_step
    StepStreams ss;
};

struct lbm_group {
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    lbm_allocator alloc_copy{};
    DeviceMem mem;
    std::vector<lbm_run *> members;
    bool dirty = true;
    int storage = -1;
    const KernelSet *ks = nullptr;    // stencil of the members (set by the first member)
    lbm_launch launch{64, 4, 32, 2, -1};
    hipGraphExec_t graph = nullptr;   // graph_G batched steps of the current membership
    int graph_G = 0;
    bool graph_failed = false;
    RunDev **druns = nullptr;
    int *dprefix = nullptr;
    long long *dlimits = nullptr;
    long long *hlimits = nullptr;     // pinned
    int *dflags = nullptr;            // lbm_group_check: one flag per member
    int *hflags = nullptr;            // pinned
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    int blocks[NCLS] = {0, 0, 0, 0};
    size_t cap = 0;
    int poison = 0;                   // some member has the NaN canary on
    bool ranges = false;              // some member asks for roctx ranges around the steps
};

namespace {

// ---- geometry ------------------------------------------------------------------------------
lbm_status setup_geometry(lbm_run *h, RunDev &R) {
    const lbm_desc &d = h->desc;
    R.Wxm = h->pml[XMIN] ? h->W : 0;
    R.Wxp = h->pml[XMAX] ? h->W : 0;
    R.Wym = h->pml[YMIN] ? h->W : 0;
    R.Wyp = h->pml[YMAX] ? h->W : 0;
    R.Nx = d.nx + R.Wxm + R.Wxp;
    R.Ny = d.ny + R.Wym + R.Wyp;
    R.W = h->W;
    for (int s = 0; s < 4; ++s) R.bc[s] = h->bc[s];
    R.pml_terms = (int)h->pml_terms;
    bool cbc_a = false;
    for (int s = 0; s < 4; ++s) cbc_a = cbc_a || h->bc[s] == BC_NRBC_A;
    // the appendix's PML moments and CBC (A) need more than the node's own state: their targets
    // are formed ahead of phase A by k_target
    R.tgt_pre = h->pml_terms != 0 || cbc_a;
    if ((h->bc[XMIN] == BC_PERIODIC) != (h->bc[XMAX] == BC_PERIODIC) ||
        (h->bc[YMIN] == BC_PERIODIC) != (h->bc[YMAX] == BC_PERIODIC))
        return fail(LBM_ERR_ARG, "periodic must be set on both sides of an axis");
    for (int s = 0; s < 4; ++s)
        if (h->pml[s] && h->W > 0 && h->bc[s] == BC_PERIODIC)
            return fail(LBM_ERR_ARG, "PML on a periodic side");
    R.open_x = h->bc[XMIN] != BC_PERIODIC;
    R.open_y = h->bc[YMIN] != BC_PERIODIC;
    if ((R.open_x && R.Nx < 7) || (R.open_y && R.Ny < 7))
        return fail(LBM_ERR_ARG, "an open axis needs at least 7 nodes (3 boundary + 1 + 3)");
    if ((!R.open_x && R.Nx < 3) || (!R.open_y && R.Ny < 3))
        return fail(LBM_ERR_ARG, "a periodic axis needs at least 3 nodes");
    if ((long long)R.Nx * R.Ny > (1LL << 30)) return fail(LBM_ERR_ARG, "grid too large");
    R.qd = std::max(h->W + 1, 3);
    int depth[4];
    for (int s = 0; s < 4; ++s) {
        int g = 3;
        if (is_char_bc(h->bc[s])) g = std::max(g, 5);
        if (h->pml[s] && h->W > 0) g = std::max(g, R.qd);
        depth[s] = g;
    }
    R.gxm = std::min(depth[XMIN], R.Nx);
    R.gxp = std::min(depth[XMAX], R.Nx - R.gxm);
    R.gym = std::min(depth[YMIN], R.Ny);
    R.gyp = std::min(depth[YMAX], R.Ny - R.gym);
    R.rxm = is_char_bc(h->bc[XMIN]) ? 3 : 0;
    R.rxp = is_char_bc(h->bc[XMAX]) ? 3 : 0;
    R.rym = is_char_bc(h->bc[YMIN]) ? 3 : 0;
    R.ryp = is_char_bc(h->bc[YMAX]) ? 3 : 0;
    R.ring_n = (R.rym + R.ryp) * R.Nx + (R.Ny - R.rym - R.ryp) * (R.rxm + R.rxp);
    R.fx0 = R.gxm; R.fx1 = R.Nx - R.gxp;
    R.fy0 = R.gym; R.fy1 = R.Ny - R.gyp;
    long long fast = (long long)std::max(0, R.fx1 - R.fx0) * std::max(0, R.fy1 - R.fy0);
    R.frame_n = (int)((long long)R.Nx * R.Ny - fast);
    // the frame off the ring: strips between the ring's inner rectangle and the fast rectangle
    // (the frame is at least as deep as the ring on every side unless the fast rectangle is
    // empty; the clamps then make the strips cover the ring's inner rectangle)
    {
        const int nxr = R.Nx - R.rxm - R.rxp, nyr = R.Ny - R.rym - R.ryp;
        R.axm = std::min(std::max(R.gxm - R.rxm, 0), nxr);
        R.axp = std::min(std::max(R.gxp - R.rxp, 0), nxr - R.axm);
        R.aym = std::min(std::max(R.gym - R.rym, 0), nyr);
        R.ayp = std::min(std::max(R.gyp - R.ryp, 0), nyr - R.aym);
        const long long ann = (long long)(R.aym + R.ayp) * nxr +
                              (long long)(nyr - R.aym - R.ayp) * (R.axm + R.axp);
        if (ann != (long long)R.frame_n - R.ring_n)
            return fail(LBM_ERR_UNSUPPORTED, "frame numbering: the annulus does not cover the frame");
        R.ann_n = (int)ann;
        R.ann0 = (int)round_up(R.ring_n, 64);
    }
    R.has_q = h->W > 0 && (h->pml[0] || h->pml[1] || h->pml[2] || h->pml[3]);
    // Padding each population row past the 64-element rounding staggers the 74 row streams of a
    // bulk tile across HBM channels: +4% bulk bandwidth at 4224^2 in FP64 and FP32 (64 elements);
    // FP16 measured best without it.
    const int pad = d.row_pad > 0 ? d.row_pad : d.row_pad < 0 ? 0 : (d.storage == ST_F16 ? 0 : 64);
    const long long row = round_up(R.Nx, 64) + (d.layout == 0 ? pad : 0);
    const int nq = h->lat->q;
    if (d.layout == 0) {            // rows: the q population rows of a grid row adjacent
        R.plane = row;
        R.pitch = (int)(nq * row);
        R.fsize = (long long)nq * row * R.Ny;
    } else {                        // planes: one padded plane per velocity
        R.pitch = (int)row;
        R.plane = round_up(row * R.Ny, 64);
        R.fsize = (long long)nq * R.plane;
    }
    R.qplane = round_up(std::max(R.ann0 + R.ann_n, 1), 64);
    R.rplane = round_up(std::max(R.ring_n, 1), 64);
    // the bulk kernel addresses a tile (at most 4 rows) with a 32-bit byte offset from a
    // uniform base; the frame arrays use 32-bit element indices
    if ((unsigned long long)R.qplane * 4 >= (1ULL << 31))
        return fail(LBM_ERR_ARG, "grid too large: frame arrays must stay below 4 GiB");
    for (int k = 0; k < 3; ++k) {
        int tx = 64 << k, ty = 256 / tx;
        if (fast > 0) {
            int xa = (R.fx0 / tx) * tx;
            R.tiles_x[k] = (R.fx1 - xa + tx - 1) / tx;
            R.tiles_y[k] = (R.fy1 - R.fy0 + ty - 1) / ty;
        } else {
            R.tiles_x[k] = 0;
            R.tiles_y[k] = 0;
        }
    }
    return LBM_OK;
}

// Mean-state Hermite coefficients of the equilibrium (see lbm_kernels.hip): fourth order
// (eq. feq-4) for D2Q37, third order (eq. feq-3) for D2Q17.
void fill_constants(lbm_run *h, RunDev &R) {
    const lbm_desc &d = h->desc;
    const LatticeInfo &lt = *h->lat;
    const bool o4 = lt.order == 4, o2 = lt.order == 2;
    R.storage = d.storage;
    R.omega = 1.0 / d.tau;
    R.rho0 = d.rho0; R.u0x = d.ux0; R.u0y = d.uy0; R.T0 = d.T0;
    R.th0 = d.T0 - 1.0;
    R.b0 = d.ux0 * d.ux0 + d.uy0 * d.uy0;
    R.r0x = lt.r * d.ux0; R.r0y = lt.r * d.uy0;
    R.sigma_max = h->sigma_max;
    R.inv_W2 = h->W > 0 ? 1.0 / ((double)h->W * h->W) : 0.0;
    const double th0 = R.th0, b0 = R.b0;
    const double k0 = o4 ? 1.0 - 0.5 * b0 - th0 + 0.125 * b0 * b0 + th0 * b0 + th0 * th0
                         : 1.0 - 0.5 * b0 - th0;
    const double k1 = 1.0 - 0.5 * b0 - 2.0 * th0;
    const double k2a = o4 ? 0.5 - 0.25 * b0 - 1.5 * th0 : 0.5;
    const double k2s = o4 ? 0.5 * th0 - 0.25 * th0 * b0 - th0 * th0 : 0.5 * th0;
    double E0[NSHELL_MAX];
    for (int s = 0; s < lt.nshell; ++s) {
        double sv = lt.r * lt.r * lt.shell_e2[s];
        E0[s] = k0 + k2s * sv + (o4 ? 0.125 * th0 * th0 * sv * sv : 0.0);
        R.E2_0[s] = k2a + (o4 ? 0.25 * th0 * sv : 0.0);
        R.O1_0[s] = o2 ? 1.0 : k1 + 0.5 * th0 * sv;   // eq. feq-2: the odd part is a itself
    }
    R.H0rest = k0;
    h->fbar[0] = lt.shell_w[0] * d.rho0 * k0;
    for (int p = 0; p < lt.npair; ++p) {
        int sh = lt.psh[p];
        double a0 = lt.pex[p] * R.r0x + lt.pey[p] * R.r0y;
        R.H0e[p] = E0[sh] + R.E2_0[sh] * a0 * a0 + (o4 ? a0 * a0 * a0 * a0 / 24.0 : 0.0);
        R.H0o[p] = o2 ? a0 : a0 * (R.O1_0[sh] + a0 * a0 / 6.0);
        h->fbar[1 + 2 * p] = lt.shell_w[sh] * d.rho0 * (R.H0e[p] + R.H0o[p]);
        h->fbar[2 + 2 * p] = lt.shell_w[sh] * d.rho0 * (R.H0e[p] - R.H0o[p]);
    }
    R.omega_f = (float)R.omega; R.rho0_f = (float)R.rho0; R.u0x_f = (float)R.u0x;
    R.u0y_f = (float)R.u0y; R.th0_f = (float)R.th0; R.b0_f = (float)R.b0;
    R.r0x_f = (float)R.r0x; R.r0y_f = (float)R.r0y; R.T0_f = (float)R.T0;
    R.H0rest_f = (float)R.H0rest;
    for (int p = 0; p < lt.npair; ++p) { R.H0e_f[p] = (float)R.H0e[p]; R.H0o_f[p] = (float)R.H0o[p]; }
    for (int s = 0; s < lt.nshell; ++s) { R.E2_0_f[s] = (float)R.E2_0[s]; R.O1_0_f[s] = (float)R.O1_0[s]; }
    R.scale = 1.0; R.inv_scale = 1.0;
}

void set_scale(RunDev &R, double s) {
    R.scale = s; R.inv_scale = 1.0 / s;
    R.scale_f = (float)s; R.inv_scale_f = (float)(1.0 / s);
}

size_t footprint_of(const RunDev &R, int storage, int nq) {
    size_t b = 2 * (size_t)R.fsize * elem_size(storage);
    if (R.has_q) b += (size_t)nq * R.qplane * compute_size(storage);
    b += 2 * 4 * (size_t)R.qplane * sizeof(double);
    if (R.ring_n > 0) b += (size_t)nq * R.rplane * compute_size(storage);
    if (R.tgt_pre && R.ring_n > 0) b += 4 * (size_t)R.rplane * sizeof(double);
    b += sizeof(RunDev) + 256 * 4 + nq * sizeof(double);
    // lbm_init_fields' transient staging of the four input fields (and, for FP16 storage, the
    // per-block maxima that choose the scale): part of the peak while the run is set up
    const size_t nn = (size_t)R.Nx * R.Ny;
    b += 4 * nn * sizeof(double) + (storage == ST_F16 ? ((nn + 255) / 256) * sizeof(float) + 256 : 0);
    return b;
}

void compute_blocks(const RunDev &R, int tx, int nb[NCLS]) {
    int k = tx_index(tx);
    nb[CLS_BULK] = R.tiles_x[k] * R.tiles_y[k];
    const int fb = frame_block_count(R.ann_n);
    const int rb = ring_block_count(R.ring_n);
    nb[CLS_FRAME] = rb + fb;
    nb[CLS_A] = rb + (R.has_q ? fb : 0);
    nb[CLS_TGT] = R.tgt_pre ? rb : 0;
}

lbm_status upload_prefix(lbm_run *h) {
    compute_blocks(h->hd, h->launch.bulk_tx, h->nblocks);
    int pre[2 * NCLS];
    for (int c = 0; c < NCLS; ++c) { pre[2 * c] = 0; pre[2 * c + 1] = h->nblocks[c]; }
    HIP_TRY(hipMemcpyAsync(h->dprefix, pre, sizeof pre, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

LaunchSet single_set(lbm_run *h) {
    LaunchSet L;
    L.ks = h->ks;
    L.runs = h->dptr;
    for (int c = 0; c < NCLS; ++c) {
        L.prefix[c] = h->dprefix + 2 * c;
        L.blocks[c] = h->nblocks[c];
    }
    L.poison = (h->debug & LBM_DEBUG_POISON) ? 1 : 0;
    L.split = h->launch.split;
    L.nruns = 1;
    return L;
}

// Fold finished timing-event pairs into the totals and return them to the pool, so the number
// of live events stays bounded by the steps in flight.
void harvest_events(lbm_run *h, bool wait) {
    size_t k = 0;
    for (; k < h->pending.size(); ++k) {
        auto &ev = h->pending[k];
        if (!wait && hipEventQuery(ev.b) != hipSuccess) break;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, ev.a, ev.b) == hipSuccess) {
            h->prof_ms[ev.cls] += t;
            h->prof_n[ev.cls] += 1;
        }
        h->pool.push_back(ev.a);
        h->pool.push_back(ev.b);
    }
    (void)hipGetLastError();
    h->pending.erase(h->pending.begin(), h->pending.begin() + k);
}

hipEvent_t take_event(lbm_run *h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Sub-step ks of a batch of steps of a launch set.  Dependencies: the characteristic targets and
// phase A (characteristic fill of the ring, Q update) before the frame kernel (grad Q reads
// neighbours' Q of the new level); the bulk kernel depends on neither; the next sub-step waits
// for everything.  With a side stream the boundary chain runs beside the bulk kernel; `fused`
// launches phase A and the bulk tiles as one grid, so the latency-bound boundary blocks run
// beside the streaming tiles on one stream (and in graphs).
// Profiling (`prof` non-null): mode 1 runs the classes in order on one stream with HIP events
// timing the bulk kernel (class 0), the frame kernel (class 1) and phase A (class 2); mode 2 keeps
// the configured schedule and times its step grid (class 0: the fused phase-A + bulk grid, or the
// bulk kernel) and the frame kernel (class 1); mode 3 does so on every fourth sub-step only.  The
// events of the kernels are attached to their dispatch (their own start and end); phase A in
// mode 1 is bracketed by event records.
lbm_status enqueue_substep(const LaunchSet &L, int storage, int tx, int ks, hipStream_t s,
                           StepStreams *ss, bool fused, lbm_run *prof) {
    const bool has_a = L.blocks[CLS_A] > 0;
    const bool has_f = L.blocks[CLS_FRAME] > 0;
    const bool has_b = L.blocks[CLS_BULK] > 0;
    if (L.poison) HIP_TRY(L.ks->poison(L, storage, ks, s));
    const int pm = prof ? prof->prof : 0;
    const int mode = pm == 3 ? ((ks & 3) == 0 ? 2 : 0) : pm;
    hipEvent_t ev[6] = {};
    if (mode) {
        harvest_events(prof, false);
        for (int k = 0; k < 6; ++k) ev[k] = take_event(prof);
    }
    const bool classes = mode == 1;
    const bool side = ss && ss->ok && !classes;
    const bool grid = fused && !classes && !side;   // phase A and the bulk tiles in one grid
    const bool t0 = mode && (grid ? (has_a || has_b) : has_b), t1 = mode && has_f;
    hipEvent_t a0 = t0 ? ev[0] : nullptr, b0 = t0 ? ev[1] : nullptr;
    hipEvent_t a1 = t1 ? ev[2] : nullptr, b1 = t1 ? ev[3] : nullptr;
    if (grid) {
        HIP_TRY(L.ks->target(L, storage, ks, s));
        HIP_TRY(L.ks->phase_a_bulk(L, storage, tx, ks, s, a0, b0));
        HIP_TRY(L.ks->frame(L, storage, ks, s, a1, b1));
    } else if (!side) {
        if (classes && has_a) HIP_TRY(hipEventRecord(ev[4], s));
        HIP_TRY(L.ks->target(L, storage, ks, s));
        HIP_TRY(L.ks->phase_a(L, storage, ks, s));
        if (classes && has_a) HIP_TRY(hipEventRecord(ev[5], s));
        HIP_TRY(L.ks->frame(L, storage, ks, s, a1, b1));
        HIP_TRY(L.ks->bulk(L, storage, tx, ks, s, a0, b0));
    } else {
        HIP_TRY(hipEventRecord(ss->fork, s));
        HIP_TRY(hipStreamWaitEvent(ss->side, ss->fork, 0));
        HIP_TRY(L.ks->target(L, storage, ks, ss->side));
        HIP_TRY(L.ks->phase_a(L, storage, ks, ss->side));
        HIP_TRY(L.ks->frame(L, storage, ks, ss->side, a1, b1));
        HIP_TRY(hipEventRecord(ss->done, ss->side));
        HIP_TRY(L.ks->bulk(L, storage, tx, ks, s, a0, b0));
        HIP_TRY(hipStreamWaitEvent(s, ss->done, 0));
    }
    if (mode) {
        const bool used[3] = {t0, t1, classes && has_a};
        for (int c = 0; c < 3; ++c) {
            if (used[c]) prof->pending.push_back({ev[2 * c], ev[2 * c + 1], c});
            else { prof->pool.push_back(ev[2 * c]); prof->pool.push_back(ev[2 * c + 1]); }
        }
    }
    return LBM_OK;
}

// A batch of nb sub-steps, then one launch that advances every run's step counter and buffer
// parity by the sub-steps it was active for.
lbm_status enqueue_batch(const LaunchSet &L, int storage, int tx, int nb, hipStream_t s,
                         StepStreams *ss, bool fused, lbm_run *prof) {
    for (int ks = 0; ks < nb; ++ks) {
        lbm_status st = enqueue_substep(L, storage, tx, ks, s, ss, fused, prof);
        if (st != LBM_OK) return st;
    }
    HIP_TRY(L.ks->advance(L, nb, s));
    return LBM_OK;
}

// Sub-steps per eager batch when graphs are off.
constexpr int EAGER_BATCH = 32;

void drop_graph(lbm_run *h) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    h->graph_G = 0;
}

// Capture G in-order steps of a launch set on stream s into an executable graph; nullptr if the
// runtime refuses (the caller then launches eagerly).
hipGraphExec_t capture_steps(const LaunchSet &L, int storage, int tx, bool fused, hipStream_t s, int G) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    lbm_status st = enqueue_batch(L, storage, tx, G, s, nullptr, fused, nullptr);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != LBM_OK || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return nullptr;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return x;
}

lbm_status build_graph(lbm_run *h, int G) {
    drop_graph(h);
    h->graph = capture_steps(single_set(h), h->desc.storage, h->launch.bulk_tx, h->launch.overlap == 2,
                             h->stream, G);
    if (!h->graph) {
        h->graph_failed = true;
        return LBM_OK;
    }
    h->graph_G = G;
    h->graph_tx = h->launch.bulk_tx;
    h->graph_ov = h->launch.overlap;
    h->graph_split = h->launch.split;
    return LBM_OK;
}

bool finite_all(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ULL; }
    return h;
}

// Refresh the host copy of the device-updated fields (par, step, limit).
lbm_status pull_state(lbm_run *h) {
    RunDev tmp;
    HIP_TRY(hipMemcpyAsync(&tmp, h->dd, sizeof(RunDev), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->hd.par = tmp.par;
    h->hd.step = tmp.step;
    h->hd.limit = tmp.limit;
    return LBM_OK;
}

}  // namespace

// ============================================================================================
// C ABI
// ============================================================================================
extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_velocities(int32_t lattice, int32_t *e, double *w, double *r) {
    const LatticeInfo *li = lattice_info(lattice);
    if (!li) return fail(LBM_ERR_ARG, "lattice must be 37, 17 or 9");
    const LatticeInfo &lt = *li;
    for (int i = 0; i < lt.q; ++i) {
        if (e) { e[2 * i] = lt.ex(i); e[2 * i + 1] = lt.ey(i); }
        if (w) w[i] = lt.shell_w[lt.shell(i)];
    }
    if (r) *r = lt.r;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_desc *desc, lbm_handle *out) {
    if (!desc || !out) return fail(LBM_ERR_ARG, "NULL argument");
    *out = nullptr;
    const lbm_desc &d = *desc;
    if (d.nx < 1 || d.ny < 1) return fail(LBM_ERR_ARG, "bulk size must be >= 1");
    if (!(d.tau > 0.5) || !std::isfinite(d.tau)) return fail(LBM_ERR_ARG, "tau must be > 0.5");
    if (!std::isfinite(d.rho0) || !std::isfinite(d.ux0) || !std::isfinite(d.uy0) ||
        !std::isfinite(d.T0) || !(d.rho0 > 0) || !(d.T0 > 0))
        return fail(LBM_ERR_ARG, "mean state must be finite with rho0 > 0 and T0 > 0");
    if (d.storage < LBM_F64 || d.storage > LBM_F16_DEV) return fail(LBM_ERR_ARG, "unknown storage");
    if (d.layout != 0 && d.layout != 1) return fail(LBM_ERR_ARG, "unknown layout");
    if (d.row_pad < -1 || d.row_pad > 4096) return fail(LBM_ERR_ARG, "row_pad must be in -1..4096");
    if (!lattice_info(d.lattice)) return fail(LBM_ERR_ARG, "lattice must be 37, 17 or 9");
    if (d.storage == LBM_F16_DEV && d.f16_scale != 0.0) {
        int ex;
        double m = std::frexp(d.f16_scale, &ex);
        if (!(d.f16_scale > 0) || m != 0.5) return fail(LBM_ERR_ARG, "f16_scale must be a power of two");
    }
    lbm_run *h = new lbm_run();
    h->desc = d;
    h->lat = lattice_info(d.lattice);
    h->desc.lattice = h->lat->q;
    h->ks = h->lat->q == 17 ? &k17::kernels : h->lat->q == 9 ? &k9::kernels : &k37::kernels;
    if (d.allocator) {
        h->alloc_copy = *d.allocator;
        h->desc.allocator = &h->alloc_copy;
        h->mem.alloc = &h->alloc_copy;
    }
    *out = h;
    return LBM_OK;
}

lbm_status lbm_set_pml(lbm_handle h, unsigned mask, int32_t W, double sigma_max) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (h->inited) return fail(LBM_ERR_STATE, "configure before lbm_init_fields");
    if (W < 0 || !(sigma_max >= 0) || !std::isfinite(sigma_max)) return fail(LBM_ERR_ARG, "W >= 0 and finite sigma_max >= 0 required");
    if (mask & ~15u) return fail(LBM_ERR_ARG, "bad side mask");
    h->W = W;
    h->sigma_max = sigma_max;
    for (int s = 0; s < 4; ++s) h->pml[s] = (mask >> s) & 1u;
    return LBM_OK;
}

lbm_status lbm_set_bc(lbm_handle h, unsigned mask, lbm_bc kind) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (h->inited) return fail(LBM_ERR_STATE, "configure before lbm_init_fields");
    // A C caller may pass any int; C++ may not load an enum outside its enumerators' range, so
    // the value is read as the int it was passed as.
    int k;
    static_assert(sizeof k == sizeof kind, "lbm_bc is passed as an int");
    std::memcpy(&k, &kind, sizeof k);
    if (k < LBM_BC_PERIODIC || k > LBM_BC_NRBC_A) return fail(LBM_ERR_ARG, "unknown boundary kind");
    if (mask & ~15u) return fail(LBM_ERR_ARG, "bad side mask");
    for (int s = 0; s < 4; ++s)
        if ((mask >> s) & 1u) h->bc[s] = k;
    return LBM_OK;
}

lbm_status lbm_set_nrbc_pml_terms(lbm_handle h, unsigned flags) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (h->inited) return fail(LBM_ERR_STATE, "configure before lbm_init_fields");
    if (flags & ~7u) return fail(LBM_ERR_ARG, "PML term flags must be a subset of bits 0..2");
    h->pml_terms = flags;
    return LBM_OK;
}

lbm_status lbm_set_debug(lbm_handle h, unsigned flags) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (flags & ~(unsigned)(LBM_DEBUG_POISON | LBM_DEBUG_RANGES)) return fail(LBM_ERR_ARG, "unknown debug flag");
    if (h->debug == flags) return LBM_OK;
    h->debug = flags;
    drop_graph(h);                       // captured steps are recaptured with the new flags
    if (h->group) h->group->dirty = true;
    return LBM_OK;
}

lbm_status lbm_grid(lbm_handle h, int32_t *Nx, int32_t *Ny) {
    if (!h || !Nx || !Ny) return fail(LBM_ERR_ARG, "NULL argument");
    int wx = (h->pml[XMIN] ? h->W : 0) + (h->pml[XMAX] ? h->W : 0);
    int wy = (h->pml[YMIN] ? h->W : 0) + (h->pml[YMAX] ? h->W : 0);
    *Nx = h->desc.nx + wx;
    *Ny = h->desc.ny + wy;
    return LBM_OK;
}

lbm_status lbm_footprint(lbm_handle h, size_t *bytes) {
    if (!h || !bytes) return fail(LBM_ERR_ARG, "NULL argument");
    RunDev R{};
    lbm_status st = setup_geometry(h, R);
    if (st != LBM_OK) return st;
    *bytes = footprint_of(R, h->desc.storage, h->lat->q);
    return LBM_OK;
}

lbm_status lbm_node_classes(lbm_handle h, int64_t out[4]) {
    if (!h || !out) return fail(LBM_ERR_ARG, "NULL argument");
    RunDev R{};
    lbm_status st = setup_geometry(h, R);
    if (st != LBM_OK) return st;
    out[0] = (int64_t)std::max(0, R.fx1 - R.fx0) * std::max(0, R.fy1 - R.fy0);
    out[1] = R.frame_n;
    int64_t q = 0;
    if (R.has_q)
        for (int y = 0; y < R.Ny; ++y)
            for (int x = 0; x < R.Nx; ++x)
                q += (R.Wxm > 0 && x < R.qd) || (R.Wxp > 0 && x >= R.Nx - R.qd) ||
                     (R.Wym > 0 && y < R.qd) || (R.Wyp > 0 && y >= R.Ny - R.qd);
    out[2] = q;
    out[3] = R.ring_n;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_handle h, const double *rho, const double *ux, const double *uy,
                           const double *T) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (h->inited) return fail(LBM_ERR_STATE, "already initialised");
    if (!rho || !ux || !uy || !T) return fail(LBM_ERR_ARG, "NULL field");
    RunDev R{};
    lbm_status st = setup_geometry(h, R);
    if (st != LBM_OK) return st;
    const size_t nn = (size_t)R.Nx * R.Ny;
    if (!finite_all(rho, nn) || !finite_all(ux, nn) || !finite_all(uy, nn) || !finite_all(T, nn))
        return fail(LBM_ERR_ARG, "non-finite initial field");
    for (size_t i = 0; i < nn; ++i)
        if (!(rho[i] > 0) || !(T[i] > 0)) return fail(LBM_ERR_ARG, "initial rho and T must be > 0");
    fill_constants(h, R);
    if (h->desc.stream) {
        h->stream = (hipStream_t)h->desc.stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
        h->stream = h->own_stream;
    }
    const int storage = h->desc.storage;
    const size_t es = elem_size(storage), cs = compute_size(storage);
    h->footprint = footprint_of(R, storage, h->lat->q);
    for (int b = 0; b < 2; ++b) {
        R.f[b] = h->mem.get((size_t)R.fsize * es);
        R.U[b] = (double *)h->mem.get(4 * (size_t)R.qplane * sizeof(double));
        if (!R.f[b] || !R.U[b]) { h->mem.release_all(); return fail(LBM_ERR_OOM, "device allocation failed"); }
    }
    R.Q = R.has_q ? h->mem.get((size_t)h->lat->q * R.qplane * cs) : nullptr;
    R.G = R.ring_n > 0 ? h->mem.get((size_t)h->lat->q * R.rplane * cs) : nullptr;
    const bool need_p = R.tgt_pre && R.ring_n > 0;
    R.P = need_p ? (double *)h->mem.get(4 * (size_t)R.rplane * sizeof(double)) : nullptr;
    h->dd = (RunDev *)h->mem.get(sizeof(RunDev));
    h->dptr = (RunDev **)h->mem.get(sizeof(RunDev *));
    h->dprefix = (int *)h->mem.get(2 * NCLS * sizeof(int));
    h->fbar_d = (double *)h->mem.get(h->lat->q * sizeof(double));
    h->dflag = (int *)h->mem.get(sizeof(int));
    if ((R.has_q && !R.Q) || (R.ring_n > 0 && !R.G) || (need_p && !R.P) || !h->dd || !h->dptr || !h->dprefix ||
        !h->fbar_d || !h->dflag) {
        h->mem.release_all();
        return fail(LBM_ERR_OOM, "device allocation failed");
    }
    if (h->mem.overlapping()) {
        h->mem.release_all();
        return fail(LBM_ERR_ARG, "device buffers overlap: the allocator returned aliasing memory");
    }
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipMemsetAsync(R.f[b], 0, (size_t)R.fsize * es, h->stream));
        HIP_TRY(hipMemsetAsync(R.U[b], 0, 4 * (size_t)R.qplane * sizeof(double), h->stream));
    }
    if (R.Q) HIP_TRY(hipMemsetAsync(R.Q, 0, (size_t)h->lat->q * R.qplane * cs, h->stream));
    if (R.G) HIP_TRY(hipMemsetAsync(R.G, 0, (size_t)h->lat->q * R.rplane * cs, h->stream));
    if (R.P) HIP_TRY(hipMemsetAsync(R.P, 0, 4 * (size_t)R.rplane * sizeof(double), h->stream));
    R.par = 0; R.step = 0; R.limit = 0;
    set_scale(R, 1.0);
    if (storage == ST_F16 && h->desc.f16_scale > 0) set_scale(R, h->desc.f16_scale);
    h->hd = R;
    HIP_TRY(hipMemcpyAsync(h->dd, &h->hd, sizeof(RunDev), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->dptr, &h->dd, sizeof(RunDev *), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->fbar_d, h->fbar, h->lat->q * sizeof(double), hipMemcpyHostToDevice, h->stream));
    // fields to the device
    double *dfield = (double *)h->mem.get(4 * nn * sizeof(double));
    if (!dfield) { h->mem.release_all(); return fail(LBM_ERR_OOM, "device allocation failed"); }
    if (h->mem.overlapping()) {
        h->mem.release_all();
        return fail(LBM_ERR_ARG, "device buffers overlap: the allocator returned aliasing memory");
    }
    const double *src[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
        HIP_TRY(hipMemcpyAsync(dfield + k * nn, src[k], nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (storage == ST_F16 && !(h->desc.f16_scale > 0)) {
        // Per-run power-of-two scale: the largest initial deviation maps to about 2^10, leaving
        // 2^5 headroom below the float16 maximum for growth.
        int nb = (int)((nn + 255) / 256);
        float *dmax = (float *)h->mem.get(nb * sizeof(float));
        if (!dmax) { h->mem.release_all(); return fail(LBM_ERR_OOM, "device allocation failed"); }
        HIP_TRY(h->ks->init(h->dd, storage, R.Nx, R.Ny, dfield, dfield + nn, dfield + 2 * nn,
                            dfield + 3 * nn, dmax, h->stream));
        std::vector<float> hm(nb);
        HIP_TRY(hipMemcpyAsync(hm.data(), dmax, nb * sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->mem.put(dmax);
        float m = 0.0f;
        for (float v : hm) m = std::max(m, v);
        double s = m > 0 ? std::ldexp(1.0, (int)std::floor(std::log2(1024.0 / m))) : std::ldexp(1.0, 20);
        s = std::min(std::max(s, std::ldexp(1.0, -10)), std::ldexp(1.0, 60));
        set_scale(h->hd, s);
        HIP_TRY(hipMemcpyAsync(h->dd, &h->hd, sizeof(RunDev), hipMemcpyHostToDevice, h->stream));
    }
    HIP_TRY(h->ks->init(h->dd, storage, R.Nx, R.Ny, dfield, dfield + nn, dfield + 2 * nn, dfield + 3 * nn,
                        nullptr, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->mem.put(dfield);
    lbm_status ps = upload_prefix(h);
    if (ps != LBM_OK) return ps;
    h->inited = true;
    h->steps = 0;
    return LBM_OK;
}

// Enqueue n > 0 steps of a run that is not in a group.
lbm_status enqueue_steps(lbm_handle h, int64_t n) {
    HIP_TRY(h->ks->set_limit(h->dd, (long long)(h->steps + n), h->stream));
    LaunchSet L = single_set(h);
    int64_t left = n;
    const int G = h->launch.graph_steps;
    // Overlapped steps launch eagerly (stream capture stays single-stream); in-order steps
    // replay captured graphs of G steps.  The side stream is created on first use.
    if (h->launch.overlap == 1 && !h->desc.stream && !h->ss.ok) HIP_TRY(h->ss.create());
    const bool overlap = h->launch.overlap == 1 && h->ss.ok;
    const bool fused = h->launch.overlap == 2;
    if (!h->prof && !overlap && G > 0 && !h->graph_failed && n >= G) {
        if (!h->graph || h->graph_G != G || h->graph_tx != h->launch.bulk_tx ||
            h->graph_ov != h->launch.overlap || h->graph_split != h->launch.split) {
            lbm_status st = build_graph(h, G);
            if (st != LBM_OK) return st;
        }
        if (h->graph) {
            while (left >= G) {
                HIP_TRY(hipGraphLaunch(h->graph, h->stream));
                left -= G;
            }
        }
    }
    const int B = G > 0 ? G : EAGER_BATCH;
    while (left > 0) {
        const int nb = (int)std::min<int64_t>(left, B);
        lbm_status st = enqueue_batch(L, h->desc.storage, h->launch.bulk_tx, nb, h->stream,
                                      overlap ? &h->ss : nullptr, fused, h->prof ? h : nullptr);
        if (st != LBM_OK) return st;
        left -= nb;
    }
    h->steps += n;
    return LBM_OK;
}

lbm_status lbm_step(lbm_handle h, int64_t n) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    if (h->group) return fail(LBM_ERR_STATE, "run is in a group; step it with lbm_group_step");
    if (n < 0) return fail(LBM_ERR_ARG, "nsteps < 0");
    if (n == 0) return LBM_OK;
    TraceRange range((h->debug & LBM_DEBUG_RANGES) != 0, "lbm_step %lld", (long long)n);
    if (h->check_every <= 0) return enqueue_steps(h, n);
    // every check_every steps: the state scan of lbm_check, stopping at the first failure
    for (int64_t left = n; left > 0;) {
        const int64_t c = std::min(left, h->check_every);
        lbm_status st = enqueue_steps(h, c);
        if (st != LBM_OK) return st;
        left -= c;
        st = lbm_check(h);
        if (st == LBM_ERR_UNSTABLE)
            return fail(st, "non-finite value, rho <= 0 or T <= 0 in the state after step " +
                                std::to_string(h->steps));
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

lbm_status lbm_set_check_interval(lbm_handle h, int64_t every) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (every < 0) return fail(LBM_ERR_ARG, "check interval < 0");
    h->check_every = every;
    return LBM_OK;
}

lbm_status lbm_step_count(lbm_handle h, int64_t *steps) {
    if (!h || !steps) return fail(LBM_ERR_ARG, "NULL argument");
    *steps = h->steps;
    return LBM_OK;
}

lbm_status lbm_synchronize(lbm_handle h) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (!h->inited) return LBM_OK;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// The moments of the current step re-pull from the previous buffer; ring nodes take the
// post-boundary populations of that step, which phase A left in G.
lbm_status lbm_moments(lbm_handle h, double *rho, double *ux, double *uy, double *T, unsigned flags) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    const RunDev &R = h->hd;
    const size_t nn = (size_t)R.Nx * R.Ny;
    if (flags & LBM_DEVICE_PTRS) {
        HIP_TRY(h->ks->moments(h->dd, h->desc.storage, R.Nx, R.Ny, rho, ux, uy, T, h->stream));
        return LBM_OK;
    }
    double *tmp = (double *)h->mem.get(4 * nn * sizeof(double));
    if (!tmp) return fail(LBM_ERR_OOM, "device allocation failed");
    double *d[4] = {tmp, tmp + nn, tmp + 2 * nn, tmp + 3 * nn};
    double *o[4] = {rho, ux, uy, T};
    hipError_t e = h->ks->moments(h->dd, h->desc.storage, R.Nx, R.Ny, o[0] ? d[0] : nullptr,
                                  o[1] ? d[1] : nullptr, o[2] ? d[2] : nullptr, o[3] ? d[3] : nullptr,
                                  h->stream);
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (o[k]) e = hipMemcpyAsync(o[k], d[k], nn * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    h->mem.put(tmp);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("lbm_moments: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_populations(lbm_handle h, double *f) {
    if (!h || !f) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    const RunDev &R = h->hd;
    const size_t n = (size_t)h->lat->q * R.Nx * R.Ny;
    double *tmp = (double *)h->mem.get(n * sizeof(double));
    if (!tmp) return fail(LBM_ERR_OOM, "device allocation failed");
    hipError_t e = h->ks->export_f(h->dd, h->desc.storage, R.Nx, R.Ny, h->fbar_d, tmp, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    h->mem.put(tmp);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("lbm_populations: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_pml_q(lbm_handle h, double *Q) {
    if (!h || !Q) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    const RunDev &R = h->hd;
    const size_t n = (size_t)h->lat->q * R.Nx * R.Ny;
    if (!R.has_q) { std::memset(Q, 0, n * sizeof(double)); return LBM_OK; }
    double *tmp = (double *)h->mem.get(n * sizeof(double));
    if (!tmp) return fail(LBM_ERR_OOM, "device allocation failed");
    hipError_t e = hipMemsetAsync(tmp, 0, n * sizeof(double), h->stream);
    if (e == hipSuccess) e = h->ks->export_q(h->dd, h->desc.storage, R.ann0 + R.ann_n, tmp, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(Q, tmp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    h->mem.put(tmp);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("lbm_pml_q: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_error_norms(lbm_handle h, const double *ref_rho, const double *ref_ux,
                           const double *ref_T, double out[3]) {
    if (!h || !ref_rho || !ref_ux || !ref_T || !out) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    const RunDev &R = h->hd;
    const size_t nn = (size_t)R.Nx * R.Ny, nb = (size_t)h->desc.nx * h->desc.ny;
    const int ly = h->desc.ny;
    double *tmp = (double *)h->mem.get((3 * nn + 3 * nb + 3 * (size_t)ly + 3) * sizeof(double));
    if (!tmp) return fail(LBM_ERR_OOM, "device allocation failed");
    double *m = tmp, *refs = tmp + 3 * nn, *part = refs + 3 * nb, *dout = part + 3 * (size_t)ly;
    hipError_t e = h->ks->moments(h->dd, h->desc.storage, R.Nx, R.Ny, m, m + nn, nullptr, m + 2 * nn, h->stream);
    const double *src[3] = {ref_rho, ref_ux, ref_T};
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(refs + k * nb, src[k], nb * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = h->ks->err_rows(m, m + nn, m + 2 * nn, R.Nx, R.Wxm, R.Wym, h->desc.nx, ly, refs, refs + nb,
                            refs + 2 * nb, part, h->stream);
    if (e == hipSuccess) e = h->ks->err_final(part, ly, dout, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    h->mem.put(tmp);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("lbm_error_norms: ") + hipGetErrorString(e));
    return LBM_OK;
}

// ---- allocation-free error norms ------------------------------------------------------------
// Per-row partial sums of lbm_error_norms_noalloc: 3 doubles per bulk row.  One copy per device,
// held until the process ends; every call on a device shares it.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels take the address scratch_address returns.
constexpr int NOALLOC_MAX_ROWS = 16384;
static __device__ __align__(256) double scratch[3 * NOALLOC_MAX_ROWS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per device.
lbm_status scratch_address(double **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        double *p = nullptr;
        HIP_TRY(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LBM_ERR_DEVICE, "no device address for the scratch array");
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

lbm_status lbm_error_norms_noalloc(lbm_handle h, const double *ref_rho, const double *ref_ux,
                                   const double *ref_T, double *out) {
    if (!h || !ref_rho || !ref_ux || !ref_T || !out) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    const int ly = h->desc.ny;
    if (ly > NOALLOC_MAX_ROWS)
        return fail(LBM_ERR_ARG, "lbm_error_norms_noalloc: the bulk has " + std::to_string(ly) +
                                     " rows; its scratch holds at most " +
                                     std::to_string(NOALLOC_MAX_ROWS));
    double *part = nullptr;
    lbm_status st = scratch_address(&part);
    if (st != LBM_OK) return st;
    const RunDev &R = h->hd;
    HIP_TRY(h->ks->err_rows_state(h->dd, h->desc.storage, R.Wxm, R.Wym, h->desc.nx, ly, ref_rho, ref_ux,
                                  ref_T, part, h->stream));
    HIP_TRY(h->ks->err_final(part, ly, out, h->stream));
    return LBM_OK;
}

int32_t lbm_build_flags(void) {
#ifdef LBM_BOUNDS
    return LBM_BUILD_BOUNDS;
#else
    return 0;
#endif
}

lbm_status lbm_check(lbm_handle h) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    int *flag = h->dflag;
    int hf = 0;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = h->ks->check(h->dd, h->desc.storage, h->hd.Nx, h->hd.Ny, flag, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(LBM_ERR_DEVICE, std::string("lbm_check: ") + hipGetErrorString(e));
    if (hf & 2) return fail(LBM_ERR_DEVICE, "a kernel met an index out of range (bounds-checked build)");
    if (hf) return fail(LBM_ERR_UNSTABLE, "non-finite value, rho <= 0 or T <= 0 in the state");
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_handle h, const lbm_launch *cfg) {
    if (!h || !cfg) return fail(LBM_ERR_ARG, "NULL argument");
    if (!(cfg->bulk_tx == 64 || cfg->bulk_tx == 128 || cfg->bulk_tx == 256) ||
        cfg->bulk_tx * cfg->bulk_ty != 256)
        return fail(LBM_ERR_ARG, "bulk tile must be 64x4, 128x2 or 256x1");
    if (cfg->graph_steps < 0 || (cfg->graph_steps & 1)) return fail(LBM_ERR_ARG, "graph_steps must be even and >= 0");
    if (cfg->overlap < 0 || cfg->overlap > 2) return fail(LBM_ERR_ARG, "overlap must be 0, 1 or 2");
    if (cfg->split < -1 || cfg->split > 8) return fail(LBM_ERR_ARG, "split must be -1 or 0..8");
    if (h->group) return fail(LBM_ERR_STATE, "run is in a group");
    h->launch = *cfg;
    if (h->inited) return upload_prefix(h);
    return LBM_OK;
}

lbm_status lbm_get_launch(lbm_handle h, lbm_launch *cfg) {
    if (!h || !cfg) return fail(LBM_ERR_ARG, "NULL argument");
    *cfg = h->launch;
    return LBM_OK;
}

lbm_status lbm_profile(lbm_handle h, int enable) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (enable < 0 || enable > 3) return fail(LBM_ERR_ARG, "profile mode must be 0, 1, 2 or 3");
    h->prof = enable;
    return LBM_OK;
}

lbm_status lbm_profile_read(lbm_handle h, double ms[3], int64_t launches[3], int reset) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (h->inited) HIP_TRY(hipStreamSynchronize(h->stream));
    harvest_events(h, true);
    for (int k = 0; k < 3; ++k) {
        if (ms) ms[k] = h->prof_ms[k];
        if (launches) launches[k] = h->prof_n[k];
        if (reset) { h->prof_ms[k] = 0; h->prof_n[k] = 0; }
    }
    return LBM_OK;
}

void lbm_destroy(lbm_handle h) {
    if (!h) return;
    if (h->group) lbm_group_remove(h->group, h);
    if (h->inited) (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    for (auto &ev : h->pending) { (void)hipEventDestroy(ev.a); (void)hipEventDestroy(ev.b); }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    h->mem.release_all();
    h->ss.destroy();
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
}

// ---- checkpoint -----------------------------------------------------------------------------
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, Nx, Ny, storage, W, pml[4], bc[4], par, layout, lattice, pml_terms, pad_;
    int64_t steps, plane, qplane;
    double tau, rho0, ux0, uy0, T0, sigma_max, scale;
    uint64_t checksum;
};
}  // namespace

lbm_status lbm_save(lbm_handle h, const char *path) {
    if (!h || !path) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    lbm_status st = pull_state(h);
    if (st != LBM_OK) return st;
    const RunDev &R = h->hd;
    const int storage = h->desc.storage;
    size_t fb = (size_t)R.fsize * elem_size(storage);
    size_t qb = R.has_q ? (size_t)h->lat->q * R.qplane * compute_size(storage) : 0;
    size_t ub = 4 * (size_t)R.qplane * sizeof(double);
    size_t gb = R.ring_n > 0 ? (size_t)h->lat->q * R.rplane * compute_size(storage) : 0;
    std::vector<char> buf(2 * fb + qb + 2 * ub + gb);
    char *p = buf.data();
    for (int b = 0; b < 2; ++b) { HIP_TRY(hipMemcpy(p, R.f[b], fb, hipMemcpyDeviceToHost)); p += fb; }
    if (qb) { HIP_TRY(hipMemcpy(p, R.Q, qb, hipMemcpyDeviceToHost)); p += qb; }
    for (int b = 0; b < 2; ++b) { HIP_TRY(hipMemcpy(p, R.U[b], ub, hipMemcpyDeviceToHost)); p += ub; }
    if (gb) { HIP_TRY(hipMemcpy(p, R.G, gb, hipMemcpyDeviceToHost)); p += gb; }
    CkptHeader hdr{};
    std::memcpy(hdr.magic, "LBMPML05", 8);
    hdr.version = 5; hdr.Nx = R.Nx; hdr.Ny = R.Ny; hdr.storage = storage; hdr.W = h->W;
    hdr.layout = h->desc.layout; hdr.lattice = h->lat->q; hdr.pml_terms = (int32_t)h->pml_terms;
    for (int s = 0; s < 4; ++s) { hdr.pml[s] = h->pml[s]; hdr.bc[s] = h->bc[s]; }
    hdr.par = R.par; hdr.steps = h->steps; hdr.plane = R.plane; hdr.qplane = R.qplane;
    hdr.tau = h->desc.tau; hdr.rho0 = h->desc.rho0; hdr.ux0 = h->desc.ux0; hdr.uy0 = h->desc.uy0;
    hdr.T0 = h->desc.T0; hdr.sigma_max = h->sigma_max; hdr.scale = R.scale;
    hdr.checksum = fnv1a(buf.data(), buf.size(), 1469598103934665603ULL);
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(LBM_ERR_ARG, std::string("cannot open ") + path);
    bool ok = std::fwrite(&hdr, sizeof hdr, 1, fp) == 1 && std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(LBM_ERR_ARG, std::string("write failed: ") + path);
    return LBM_OK;
}

lbm_status lbm_load(lbm_handle h, const char *path) {
    if (!h || !path) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "initialise the handle before lbm_load");
    if (h->group) return fail(LBM_ERR_STATE, "run is in a group");
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return fail(LBM_ERR_ARG, std::string("cannot open ") + path);
    CkptHeader hdr{};
    if (std::fread(&hdr, sizeof hdr, 1, fp) != 1 || std::memcmp(hdr.magic, "LBMPML05", 8) != 0) {
        std::fclose(fp);
        return fail(LBM_ERR_ARG, "not a checkpoint file");
    }
    RunDev &R = h->hd;
    const int storage = h->desc.storage;
    bool same = hdr.Nx == R.Nx && hdr.Ny == R.Ny && hdr.storage == storage && hdr.W == h->W &&
                hdr.layout == h->desc.layout && hdr.lattice == h->lat->q &&
                hdr.plane == R.plane && hdr.qplane == R.qplane && hdr.tau == h->desc.tau &&
                hdr.rho0 == h->desc.rho0 && hdr.ux0 == h->desc.ux0 && hdr.uy0 == h->desc.uy0 &&
                hdr.T0 == h->desc.T0 && hdr.sigma_max == h->sigma_max &&
                hdr.pml_terms == (int32_t)h->pml_terms;
    for (int s = 0; s < 4; ++s) same = same && hdr.pml[s] == h->pml[s] && hdr.bc[s] == h->bc[s];
    if (!same) { std::fclose(fp); return fail(LBM_ERR_ARG, "checkpoint configuration differs from the handle's"); }
    size_t fb = (size_t)R.fsize * elem_size(storage);
    size_t qb = R.has_q ? (size_t)h->lat->q * R.qplane * compute_size(storage) : 0;
    size_t ub = 4 * (size_t)R.qplane * sizeof(double);
    size_t gb = R.ring_n > 0 ? (size_t)h->lat->q * R.rplane * compute_size(storage) : 0;
    std::vector<char> buf(2 * fb + qb + 2 * ub + gb);
    bool ok = std::fread(buf.data(), 1, buf.size(), fp) == buf.size();
    std::fclose(fp);
    if (!ok) return fail(LBM_ERR_ARG, "truncated checkpoint");
    if (fnv1a(buf.data(), buf.size(), 1469598103934665603ULL) != hdr.checksum)
        return fail(LBM_ERR_ARG, "checkpoint checksum mismatch");
    HIP_TRY(hipStreamSynchronize(h->stream));
    char *p = buf.data();
    for (int b = 0; b < 2; ++b) { HIP_TRY(hipMemcpy(R.f[b], p, fb, hipMemcpyHostToDevice)); p += fb; }
    if (qb) { HIP_TRY(hipMemcpy(R.Q, p, qb, hipMemcpyHostToDevice)); p += qb; }
    for (int b = 0; b < 2; ++b) { HIP_TRY(hipMemcpy(R.U[b], p, ub, hipMemcpyHostToDevice)); p += ub; }
    if (gb) { HIP_TRY(hipMemcpy(R.G, p, gb, hipMemcpyHostToDevice)); p += gb; }
    R.par = hdr.par;
    R.step = hdr.steps;
    R.limit = hdr.steps;
    set_scale(R, hdr.scale);
    HIP_TRY(hipMemcpy(h->dd, &R, sizeof(RunDev), hipMemcpyHostToDevice));
    h->steps = hdr.steps;
    return LBM_OK;
}

// ---- autotune -------------------------------------------------------------------------------
lbm_status lbm_autotune(lbm_handle h, int32_t steps, const char *cache_path, lbm_launch *chosen) {
    if (!h) return fail(LBM_ERR_ARG, "NULL handle");
    if (!h->inited) return fail(LBM_ERR_STATE, "not initialised");
    if (h->group) return fail(LBM_ERR_STATE, "run is in a group");
    if (steps < 1) steps = 10;
    const RunDev &R = h->hd;
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "r");
        if (fp) {
            char line[256];
            while (std::fgets(line, sizeof line, fp)) {
                int nx, ny, st, q, tx, ov, sp = -1;
                if (std::sscanf(line, "%d %d %d %d %d %d %d", &nx, &ny, &st, &q, &tx, &ov, &sp) < 6) continue;
                if (nx == R.Nx && ny == R.Ny && st == h->desc.storage && q == h->lat->q) {
                    std::fclose(fp);
                    lbm_launch c = h->launch;
                    c.bulk_tx = tx; c.bulk_ty = 256 / tx; c.overlap = ov; c.split = sp;
                    lbm_status s2 = lbm_set_launch(h, &c);
                    if (chosen) *chosen = h->launch;
                    return s2;
                }
            }
            std::fclose(fp);
        }
    }
    // scratch run with the same geometry at the mean state, on a stream of the same kind
    lbm_desc d = h->desc;
    lbm_handle s = nullptr;
    lbm_status st = lbm_create(&d, &s);
    if (st != LBM_OK) return st;
    s->W = h->W; s->sigma_max = h->sigma_max; s->pml_terms = h->pml_terms;
    for (int k = 0; k < 4; ++k) { s->pml[k] = h->pml[k]; s->bc[k] = h->bc[k]; }
    const size_t nn = (size_t)R.Nx * R.Ny;
    std::vector<double> f1(nn, d.rho0), f2(nn, d.ux0), f3(nn, d.uy0), f4(nn, d.T0);
    st = lbm_init_fields(s, f1.data(), f2.data(), f3.data(), f4.data());
    if (st != LBM_OK) { lbm_destroy(s); return st; }
    int best_tx = h->launch.bulk_tx, best_ov = h->launch.overlap, best_sp = h->launch.split;
    float best = 1e30f;
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    // tile widths x schedules, and for the fused grid the phase-A placement in eighths of the tiles
    for (int ov = 0; ov < 3; ++ov) {
        if (ov == 1 && d.stream) continue;   // the side stream needs a stream the run owns
        for (int tx : {64, 128, 256}) {
            for (int sp : {0, 2, 4, 6, 8}) {
                if (ov != 2 && sp != 0) continue;
                lbm_launch c{tx, 256 / tx, 0, ov, ov == 2 ? sp : -1};
                if (lbm_set_launch(s, &c) != LBM_OK) continue;
                lbm_step(s, 2);
                (void)hipEventRecord(a, s->stream);
                lbm_step(s, steps);
                (void)hipEventRecord(b, s->stream);
                (void)hipEventSynchronize(b);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, a, b);
                if (ms < best) { best = ms; best_tx = tx; best_ov = ov; best_sp = c.split; }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    lbm_destroy(s);
    lbm_launch c = h->launch;
    c.bulk_tx = best_tx; c.bulk_ty = 256 / best_tx; c.overlap = best_ov; c.split = best_sp;
    st = lbm_set_launch(h, &c);
    if (st == LBM_OK && cache_path) {
        FILE *fp = std::fopen(cache_path, "a");
        if (fp) {
            std::fprintf(fp, "%d %d %d %d %d %d %d\n", R.Nx, R.Ny, h->desc.storage, h->lat->q, best_tx, best_ov,
                         best_sp);
            std::fclose(fp);
        }
    }
    if (chosen) *chosen = h->launch;
    return st;
}

// ---- groups ---------------------------------------------------------------------------------
lbm_status lbm_group_create(void *stream, const lbm_allocator *allocator, lbm_group_handle *out) {
    if (!out) return fail(LBM_ERR_ARG, "NULL argument");
    lbm_group *g = new lbm_group();
    if (allocator) { g->alloc_copy = *allocator; g->mem.alloc = &g->alloc_copy; }
    if (stream) g->stream = (hipStream_t)stream;
    else {
        if (hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return fail(LBM_ERR_DEVICE, "hipStreamCreate failed");
        }
        g->stream = g->own_stream;
    }
    if (hipHostMalloc((void **)&g->hlimits, 4096 * sizeof(long long), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->hflags, 4096 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&g->upload_done, hipEventDisableTiming) != hipSuccess) {
        if (g->hlimits) (void)hipHostFree(g->hlimits);
        if (g->hflags) (void)hipHostFree(g->hflags);
        if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
        delete g;
        return fail(LBM_ERR_DEVICE, "group setup failed");
    }
    *out = g;
    return LBM_OK;
}

lbm_status lbm_group_add(lbm_group_handle g, lbm_handle h) {
    if (!g || !h) return fail(LBM_ERR_ARG, "NULL argument");
    if (!h->inited) return fail(LBM_ERR_STATE, "initialise the run before adding it");
    if (h->group) return fail(LBM_ERR_STATE, "run already in a group");
    if (g->storage >= 0 && g->storage != h->desc.storage) return fail(LBM_ERR_ARG, "all runs of a group share one storage");
    if (g->ks && g->ks != h->ks) return fail(LBM_ERR_ARG, "all runs of a group share one velocity stencil");
    if (g->members.size() >= 4096) return fail(LBM_ERR_ARG, "group full (4096 runs)");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->storage = h->desc.storage;
    g->ks = h->ks;
    g->members.push_back(h);
    h->group = g;
    h->stream = g->stream;
    g->dirty = true;
    return LBM_OK;
}

lbm_status lbm_group_remove(lbm_group_handle g, lbm_handle h) {
    if (!g || !h) return fail(LBM_ERR_ARG, "NULL argument");
    auto it = std::find(g->members.begin(), g->members.end(), h);
    if (it == g->members.end()) return fail(LBM_ERR_ARG, "run is not in this group");
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->members.erase(it);
    h->group = nullptr;
    h->stream = h->own_stream ? h->own_stream : (hipStream_t)h->desc.stream;
    if (g->members.empty()) { g->storage = -1; g->ks = nullptr; }
    g->dirty = true;
    return LBM_OK;
}

lbm_status lbm_group_size(lbm_group_handle g, int32_t *n) {
    if (!g || !n) return fail(LBM_ERR_ARG, "NULL argument");
    *n = (int32_t)g->members.size();
    return LBM_OK;
}

lbm_status lbm_group_synchronize(lbm_group_handle g) {
    if (!g) return fail(LBM_ERR_ARG, "NULL argument");
    HIP_TRY(hipStreamSynchronize(g->stream));
    return LBM_OK;
}

static void group_drop_graph(lbm_group *g) {
    if (g->graph) (void)hipGraphExecDestroy(g->graph);
    g->graph = nullptr;
    g->graph_G = 0;
}

static lbm_status group_rebuild(lbm_group *g) {
    const size_t n = g->members.size();
    HIP_TRY(hipStreamSynchronize(g->stream));
    group_drop_graph(g);
    if (n > g->cap) {
        g->mem.put(g->druns); g->mem.put(g->dprefix); g->mem.put(g->dlimits); g->mem.put(g->dflags);
        size_t cap = std::max<size_t>(n, 64);
        g->druns = (RunDev **)g->mem.get(cap * sizeof(RunDev *));
        g->dprefix = (int *)g->mem.get(NCLS * (cap + 1) * sizeof(int));
        g->dlimits = (long long *)g->mem.get(cap * sizeof(long long));
        g->dflags = (int *)g->mem.get(cap * sizeof(int));
        if (!g->druns || !g->dprefix || !g->dlimits || !g->dflags)
            return fail(LBM_ERR_OOM, "device allocation failed");
        g->cap = cap;
    }
    std::vector<RunDev *> ptrs(n);
    std::vector<int> pre(NCLS * (g->cap + 1), 0);
    int tot[NCLS] = {0, 0, 0, 0};
    for (size_t k = 0; k < n; ++k) {
        lbm_run *h = g->members[k];
        ptrs[k] = h->dd;
        int nb[NCLS];
        compute_blocks(h->hd, g->launch.bulk_tx, nb);
        for (int c = 0; c < NCLS; ++c) { pre[c * (g->cap + 1) + k] = tot[c]; tot[c] += nb[c]; }
    }
    for (int c = 0; c < NCLS; ++c) pre[c * (g->cap + 1) + n] = tot[c];
    g->poison = 0;
    for (lbm_run *h : g->members) g->poison |= (h->debug & LBM_DEBUG_POISON) ? 1 : 0;
    g->ranges = false;
    for (lbm_run *h : g->members) g->ranges = g->ranges || (h->debug & LBM_DEBUG_RANGES);
    if (n) HIP_TRY(hipMemcpy(g->druns, ptrs.data(), n * sizeof(RunDev *), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->dprefix, pre.data(), pre.size() * sizeof(int), hipMemcpyHostToDevice));
    for (int c = 0; c < NCLS; ++c) g->blocks[c] = tot[c];
    g->dirty = false;
    return LBM_OK;
}

lbm_status lbm_group_step(lbm_group_handle g, const int64_t *steps, int64_t nsteps) {
    if (!g) return fail(LBM_ERR_ARG, "NULL argument");
    const size_t n = g->members.size();
    if (n == 0) return LBM_OK;
    if (g->dirty) {
        lbm_status st = group_rebuild(g);
        if (st != LBM_OK) return st;
    }
    int64_t K = 0;
    for (size_t k = 0; k < n; ++k) {
        int64_t s = steps ? steps[k] : nsteps;
        if (s < 0) return fail(LBM_ERR_ARG, "negative step count");
        K = std::max(K, s);
    }
    if (K == 0) return LBM_OK;
    TraceRange range(g->ranges, "lbm_group_step %zu %lld", n, (long long)K);
    if (g->upload_pending) HIP_TRY(hipEventSynchronize(g->upload_done));
    for (size_t k = 0; k < n; ++k) g->hlimits[k] = g->members[k]->steps + (steps ? steps[k] : nsteps);
    HIP_TRY(hipMemcpyAsync(g->dlimits, g->hlimits, n * sizeof(long long), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipEventRecord(g->upload_done, g->stream));
    g->upload_pending = true;
    HIP_TRY(g->ks->set_limits(g->druns, g->dlimits, (int)n, g->stream));
    LaunchSet L;
    L.ks = g->ks;
    L.runs = g->druns;
    for (int c = 0; c < NCLS; ++c) {
        L.prefix[c] = g->dprefix + c * (g->cap + 1);
        L.blocks[c] = g->blocks[c];
    }
    L.nruns = (int)n;
    L.poison = g->poison;
    L.split = g->launch.split;
    // Runs past their own count skip every kernel, so whole graphs of G batched steps serve any
    // mix of counts; the remainder is launched eagerly.
    int64_t left = K;
    const int G = g->launch.graph_steps;
    if (G > 0 && !g->graph_failed && K >= G) {
        if (!g->graph || g->graph_G != G) {
            group_drop_graph(g);
            g->graph = capture_steps(L, g->storage, g->launch.bulk_tx, g->launch.overlap == 2, g->stream, G);
            if (g->graph) g->graph_G = G;
            else g->graph_failed = true;
        }
        if (g->graph) {
            for (; left >= G; left -= G) HIP_TRY(hipGraphLaunch(g->graph, g->stream));
        }
    }
    const int B = G > 0 ? G : EAGER_BATCH;
    while (left > 0) {
        const int nb = (int)std::min<int64_t>(left, B);
        lbm_status st = enqueue_batch(L, g->storage, g->launch.bulk_tx, nb, g->stream, nullptr,
                                      g->launch.overlap == 2, nullptr);
        if (st != LBM_OK) return st;
        left -= nb;
    }
    for (size_t k = 0; k < n; ++k) g->members[k]->steps += steps ? steps[k] : nsteps;
    return LBM_OK;
}

lbm_status lbm_group_check(lbm_group_handle g, int32_t *flags) {
    if (!g) return fail(LBM_ERR_ARG, "NULL argument");
    const size_t n = g->members.size();
    if (n == 0) return LBM_OK;
    if (!flags) return fail(LBM_ERR_ARG, "NULL argument");
    if (g->dirty) {
        lbm_status st = group_rebuild(g);
        if (st != LBM_OK) return st;
    }
    HIP_TRY(hipMemsetAsync(g->dflags, 0, n * sizeof(int), g->stream));
    for (size_t k = 0; k < n; ++k) {
        lbm_run *h = g->members[k];
        HIP_TRY(h->ks->check(h->dd, h->desc.storage, h->hd.Nx, h->hd.Ny, g->dflags + k, g->stream));
    }
    HIP_TRY(hipMemcpyAsync(g->hflags, g->dflags, n * sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    for (size_t k = 0; k < n; ++k) flags[k] = g->hflags[k] & 2 ? 2 : g->hflags[k] ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_group_set_launch(lbm_group_handle g, const lbm_launch *cfg) {
    if (!g || !cfg) return fail(LBM_ERR_ARG, "NULL argument");
    if (!(cfg->bulk_tx == 64 || cfg->bulk_tx == 128 || cfg->bulk_tx == 256) ||
        cfg->bulk_tx * cfg->bulk_ty != 256)
        return fail(LBM_ERR_ARG, "bulk tile must be 64x4, 128x2 or 256x1");
    if (cfg->graph_steps < 0 || (cfg->graph_steps & 1)) return fail(LBM_ERR_ARG, "graph_steps must be even and >= 0");
    if (cfg->overlap != 0 && cfg->overlap != 2)
        return fail(LBM_ERR_ARG, "groups run on one stream (overlap 0 or 2)");
    if (cfg->split < -1 || cfg->split > 8) return fail(LBM_ERR_ARG, "split must be -1 or 0..8");
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->launch = *cfg;
    g->graph_failed = false;
    g->dirty = true;   // block counts depend on the tile width; graphs are recaptured
    return LBM_OK;
}

lbm_status lbm_group_get_launch(lbm_group_handle g, lbm_launch *cfg) {
    if (!g || !cfg) return fail(LBM_ERR_ARG, "NULL argument");
    *cfg = g->launch;
    return LBM_OK;
}

lbm_status lbm_group_autotune(lbm_group_handle g, int32_t steps, lbm_launch *chosen) {
    if (!g) return fail(LBM_ERR_ARG, "NULL argument");
    if (g->members.empty()) return fail(LBM_ERR_STATE, "empty group");
    if (steps < 1) steps = 10;
    // one scratch run at the mean state per distinct geometry among the members
    std::vector<lbm_run *> scratch;
    std::vector<std::array<long long, 12>> keys;
    lbm_status st = LBM_OK;
    for (lbm_run *h : g->members) {
        std::array<long long, 12> key{h->desc.nx, h->desc.ny, h->desc.storage, h->desc.layout, h->W,
                                      h->pml[0] | h->pml[1] << 1 | h->pml[2] << 2 | h->pml[3] << 3,
                                      h->bc[0], h->bc[1], h->bc[2], h->bc[3], (long long)h->pml_terms, 0};
        if (std::find(keys.begin(), keys.end(), key) != keys.end()) continue;
        keys.push_back(key);
        lbm_desc d = h->desc;
        d.stream = (void *)g->stream;
        lbm_handle s = nullptr;
        st = lbm_create(&d, &s);
        if (st != LBM_OK) break;
        scratch.push_back(s);
        s->W = h->W; s->sigma_max = h->sigma_max; s->pml_terms = h->pml_terms;
        for (int k = 0; k < 4; ++k) { s->pml[k] = h->pml[k]; s->bc[k] = h->bc[k]; }
        const size_t nn = (size_t)(h->hd.Nx) * h->hd.Ny;
        std::vector<double> f1(nn, d.rho0), f2(nn, d.ux0), f3(nn, d.uy0), f4(nn, d.T0);
        st = lbm_init_fields(s, f1.data(), f2.data(), f3.data(), f4.data());
        if (st != LBM_OK) break;
    }
    lbm_launch best_c = g->launch;
    if (st == LBM_OK) {
        lbm_group_handle sg = nullptr;
        st = lbm_group_create((void *)g->stream, g->mem.alloc, &sg);
        for (size_t k = 0; st == LBM_OK && k < scratch.size(); ++k) st = lbm_group_add(sg, scratch[k]);
        float best = 1e30f;
        hipEvent_t a = nullptr, b = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        // tile widths x {in order, fused with the phase-A blocks after 0, 2, 4, 6 or 8 eighths of
        // the tiles}
        for (int k = 0; k < 18; ++k) {
            if (st != LBM_OK) break;
            const int tx = 64 << (k % 3), j = k / 3, ov = j == 0 ? 0 : 2, sp = j == 0 ? -1 : 2 * (j - 1);
            lbm_launch c{tx, 256 / tx, 0, ov, sp};
            if ((st = lbm_group_set_launch(sg, &c)) != LBM_OK) break;
            if ((st = lbm_group_step(sg, nullptr, 2)) != LBM_OK) break;
            (void)hipEventRecord(a, g->stream);
            if ((st = lbm_group_step(sg, nullptr, steps)) != LBM_OK) break;
            (void)hipEventRecord(b, g->stream);
            (void)hipEventSynchronize(b);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) {
                best = ms; best_c = g->launch;
                best_c.bulk_tx = tx; best_c.bulk_ty = 256 / tx; best_c.overlap = ov; best_c.split = sp;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (sg) lbm_group_destroy(sg);
    }
    for (lbm_run *s : scratch) lbm_destroy(s);
    if (st != LBM_OK) return st;
    st = lbm_group_set_launch(g, &best_c);
    if (chosen) *chosen = g->launch;
    return st;
}

void lbm_group_destroy(lbm_group_handle g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    for (lbm_run *h : g->members) {
        h->group = nullptr;
        h->stream = h->own_stream ? h->own_stream : (hipStream_t)h->desc.stream;
    }
    group_drop_graph(g);
    g->mem.release_all();
    if (g->hlimits) (void)hipHostFree(g->hlimits);
    if (g->hflags) (void)hipHostFree(g->hflags);
    if (g->upload_done) (void)hipEventDestroy(g->upload_done);
    if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
    delete g;
}

}  // extern "C"
