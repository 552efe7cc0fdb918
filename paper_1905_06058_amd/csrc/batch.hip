// Batched full-range ISAM: many B-scans of uneven size (each its own nx, nk, optics and
// calibration) through the operator of Eq. 5, 13, 16, its adjoint (Eq. 17) and the FISTA
// solve of Alg. 1, with one launch per pass for each group of scans that share a kernel
// specialisation instead of one launch per pass per scan.
//
// Scans are grouped twice: by depth FFT length K = 2 nk for the NUFFT passes (whose kernels
// do not depend on nx) and by lateral length nx for the lateral passes (whose kernels do not
// depend on nk).  A launch covers all scans of a group: its workgroups are listed in a block
// map (scan, workgroup of that scan), and each scan's operands come from a record array in
// device memory.  Per-scan block counts are padded to multiples of 8 with idle entries so
// that a scan's workgroups keep the XCD placement of a single-scan launch.
//
// One FISTA iteration is the launch sequence
//   advance (t, beta) -> NUFFT forward per K group -> NUFFT adjoint per K group
//   -> update pass per nx group [-> Eq. 15 check per scan]
// whose kernels read everything that varies between calls (data pointers, step, lambda,
// weights) from the record arrays and the iteration's momentum weight from the device
// state, so the sequence is captured once in a hipGraph and replayed every iteration.
// The tuner picks each lateral group's tile width by timing the candidates.
//
// A second schedule runs FISTA as each scan's own solve (the single-scan kernels and
// launches) with the scans spread over the batch's streams, one host thread per stream, so
// that the passes of different scans overlap on the GPU where the grouped launches wait for
// the slowest scan of each pass.  The tuner times both schedules and keeps the faster one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace {

using isam::LatScan;
using isam::NuScan;
using isam::StopState;

enum LatKind { LK_C2C_FWD, LK_C2R, LK_R2C, LK_C2C_INV, LK_FISTA, LK_COUNT };
enum NuKind { NK_FWD_OP, NK_ADJ_OP, NK_FWD_FISTA, NK_ADJ_FISTA, NK_COUNT };
enum MapKind { MAP_LAT_C, MAP_LAT_R, MAP_NU_FWD, MAP_NU_ADJ };

struct BatchState {
    double t;       // FISTA t^k
    float beta;     // momentum weight of the current iteration
    int k;          // current iteration (1-based after the first advance)
    float tol;      // Eq. 15 tolerance
};

// Where a scan's partial sums live: forward NUFFT (slot 0: ||r||^2) and update pass
// (slots 0..3: Eq. 15 norms and the weighted l1 norm).
struct SumRec {
    const float* part_r;
    int nr;
    const float* part_f;
    int nf;
};

__global__ void k_batch_reset(BatchState* st, StopState* stops, int n, float tol) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->t = 1.0;
        st->beta = 0.f;
        st->k = 0;
        st->tol = tol;
    }
    if (i < n) {
        stops[i].iter = 0;
        stops[i].status = ISAM_OK;
        stops[i].rel_res = -1.0;
    }
}

// t^{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, beta_k = (t_k - 1) / t^{k+1} (Alg. 1).
__global__ void k_batch_advance(BatchState* st) {
    if (threadIdx.x == 0) {
        const double t = st->t;
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        st->beta = (float)((t - 1.0) / tn);
        st->t = tn;
        st->k += 1;
    }
}

// Eq. 15 per scan (one workgroup each), with the fixed-order FP64 sums of the single-scan
// solver; a scan that has stopped keeps its record.
__global__ __launch_bounds__(256) void k_batch_stop(const SumRec* __restrict__ recs, StopState* stops,
                                                    const BatchState* __restrict__ st) {
    const int sidx = blockIdx.x;
    if (stops[sidx].iter) return;                      // uniform
    const SumRec r = recs[sidx];
    __shared__ double sh[3][256];
    const int tid = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = tid; b < r.nf; b += 256)
        for (int i = 0; i < 3; ++i) acc[i] += r.part_f[b * isam::kRedSlots + i];
    for (int i = 0; i < 3; ++i) sh[i][tid] = acc[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int i = 0; i < 3; ++i) sh[i][tid] += sh[i][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const double d = sh[0][0], g = sh[1][0], e = sh[2][0];
        if (!isfinite(d) || !isfinite(g) || !isfinite(e)) {
            stops[sidx].status = ISAM_ENONFINITE;
            stops[sidx].iter = st->k;
        } else {
            const double rr = sqrt(d) / (fmax(sqrt(g), sqrt(e)) + 1e-12);
            stops[sidx].rel_res = rr;
            if (rr < (double)st->tol) stops[sidx].iter = st->k;
        }
    }
}

// Per scan: ||r||^2 of the last forward pass and the weighted l1 norm of z (FP64, fixed order).
__global__ __launch_bounds__(256) void k_batch_sums(const SumRec* __restrict__ recs, double* out) {
    const SumRec r = recs[blockIdx.x];
    __shared__ double sh[2][256];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < r.nr; i += 256) a += r.part_r[i * isam::kRedSlots];
    for (int i = tid; i < r.nf; i += 256) b += r.part_f[i * isam::kRedSlots + 3];
    sh[0][tid] = a;
    sh[1][tid] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            sh[0][tid] += sh[0][tid + w];
            sh[1][tid] += sh[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[2 * blockIdx.x] = sh[0][0];
        out[2 * blockIdx.x + 1] = sh[1][0];
    }
}

struct Group {
    int key;                    // K for NUFFT groups, nx for lateral groups
    std::vector<int> scans;     // batch indices
    int sel_c = 0, sel_r = 0;   // lateral tile widths requested for complex / real passes
    int map_off[2] = {0, 0};    // offsets of the group's two block maps in the map buffer
    int nblk[2] = {0, 0};       // their lengths
};

// A record array of one pass kind: host copy, device copy, pinned staging, and the event of
// its last upload (the staging area is rewritten only after that copy has run).
template <typename R>
struct Records {
    std::vector<R> host;
    R* dev = nullptr;
    R* stage = nullptr;
    hipEvent_t ev = nullptr;
    bool valid = false;         // device copy equals host copy
    int alloc(int n) {
        host.assign(n, R{});
        if (hipMalloc((void**)&dev, n * sizeof(R)) != hipSuccess) return ISAM_ENOMEM;
        if (hipHostMalloc((void**)&stage, n * sizeof(R)) != hipSuccess) return ISAM_ENOMEM;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return ISAM_EHIP;
        return ISAM_OK;
    }
    int upload(hipStream_t s) {
        if (valid && std::memcmp(stage, host.data(), host.size() * sizeof(R)) == 0) return ISAM_OK;
        if (hipEventSynchronize(ev) != hipSuccess) return ISAM_EHIP;
        std::memcpy(stage, host.data(), host.size() * sizeof(R));
        if (hipMemcpyAsync(dev, stage, host.size() * sizeof(R), hipMemcpyHostToDevice, s) != hipSuccess)
            return ISAM_EHIP;
        if (hipEventRecord(ev, s) != hipSuccess) return ISAM_EHIP;
        valid = true;
        return ISAM_OK;
    }
    void release() {
        if (dev) (void)hipFree(dev);
        if (stage) (void)hipHostFree(stage);
        if (ev) (void)hipEventDestroy(ev);
    }
};

}  // namespace

struct isam_batch_s {
    int n = 0;
    std::vector<isam_plan_t> plans;
    std::vector<int64_t> off;                 // element offsets into packed buffers (n + 1)
    std::vector<Group> nu, lat;
    int2* maps = nullptr;                     // device block maps
    int maps_cap = 0;
    Records<LatScan> latrec[LK_COUNT];
    Records<NuScan> nurec[NK_COUNT];
    Records<SumRec> sumrec;
    StopState* stops = nullptr;               // device, n
    StopState* host_stops = nullptr;          // pinned, n
    BatchState* state = nullptr;
    double* sums = nullptr;                   // device, 2n
    double* host_sums = nullptr;              // pinned, 2n
    hipStream_t cs = nullptr;                 // private stream for graph capture
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // FISTA iteration without / with Eq. 15 check
    int sched = ISAM_BATCH_SCHED_GROUPED;     // FISTA schedule
    std::vector<hipStream_t> ss;              // streams of the streams schedule (made on first use)
    std::vector<hipEvent_t> ev;               // fork event of the streams schedule
    std::vector<int> order;                   // scans by decreasing size; scan order[j] runs on ss[j % ns]
};

namespace {

using isam_batch_t = isam_batch_s*;

int lat_ntiles(const isam_plan_s* p, int sel, int real) {
    const int c = isam::lat_tile(p->nx, sel, real);
    return real ? p->nk / (2 * c) : p->nk / c;
}

// Block maps of every group for the current tile widths, uploaded synchronously (set-up only).
int build_maps(isam_batch_t b) {
    std::vector<int2> h;
    auto add = [&](Group& g, int which, auto count) {
        g.map_off[which] = (int)h.size();
        for (int i : g.scans) {
            const int nb = count(b->plans[i]);
            for (int j = 0; j < nb; ++j) h.push_back(make_int2(i, j));
            while (h.size() % 8) h.push_back(make_int2(-1, -1));     // keep XCD placement
        }
        g.nblk[which] = (int)h.size() - g.map_off[which];
    };
    for (Group& g : b->lat) {
        add(g, 0, [&](const isam_plan_s* p) { return lat_ntiles(p, g.sel_c, 0); });
        add(g, 1, [&](const isam_plan_s* p) { return lat_ntiles(p, g.sel_r, 1); });
    }
    for (Group& g : b->nu) {
        add(g, 0, [](const isam_plan_s* p) { return isam::nufft_fwd_blocks(p); });
        add(g, 1, [](const isam_plan_s* p) { return isam::nufft_adj_blocks(p); });
    }
    if ((int)h.size() > b->maps_cap) {
        if (b->maps) (void)hipFree(b->maps);
        b->maps = nullptr;
        b->maps_cap = 0;
        if (hipMalloc((void**)&b->maps, h.size() * sizeof(int2)) != hipSuccess) return ISAM_ENOMEM;
        b->maps_cap = (int)h.size();
    }
    if (hipMemcpy(b->maps, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) return ISAM_EHIP;
    return ISAM_OK;
}

// Plan-owned operands of the records (pointers into each scan's workspace, tile counts,
// twiddle tables); per-call fields are filled by the entry points.
void fill_static_records(isam_batch_t b) {
    for (const Group& g : b->lat)
        for (int i : g.scans) {
            isam_plan_s* p = b->plans[i];
            for (int k = 0; k < LK_COUNT; ++k) {
                const int real = (k == LK_C2R || k == LK_R2C);
                const int sel = real ? g.sel_r : g.sel_c;
                LatScan& r = b->latrec[k].host[i];
                r.tw = p->twX[isam::lat_radix_cap(p->nx, sel, real)];
                r.nk = p->nk;
                r.ntiles = lat_ntiles(p, sel, real);
            }
            b->latrec[LK_C2C_FWD].host[i].out = p->etahat;
            b->latrec[LK_C2R].host[i].in = p->zh;
            b->latrec[LK_R2C].host[i].out = p->rh;
            b->latrec[LK_C2C_INV].host[i].in = p->ghat;
            LatScan& f = b->latrec[LK_FISTA].host[i];
            f.out = p->fista_hat;
            f.in = p->ghat;
            f.z = p->zblk;
            f.partials = p->red.partials + (size_t)isam::nufft_fwd_blocks(p) * isam::kRedSlots;
        }
    for (int i = 0; i < b->n; ++i) {
        isam_plan_s* p = b->plans[i];
        const int rb = isam::nufft_fwd_blocks(p);
        for (int k = 0; k < NK_COUNT; ++k) {
            NuScan& r = b->nurec[k].host[i];
            r.a = p->nufft_args();
            r.nblk = (k == NK_FWD_OP || k == NK_FWD_FISTA) ? rb : isam::nufft_adj_blocks(p);
        }
        NuScan* r = b->nurec[NK_FWD_OP].host.data() + i;
        r->in = p->etahat, r->in2 = nullptr, r->out = p->zh, r->partials = nullptr;
        r = b->nurec[NK_ADJ_OP].host.data() + i;
        r->in = p->rh, r->in2 = nullptr, r->out = p->ghat, r->partials = nullptr;
        r = b->nurec[NK_FWD_FISTA].host.data() + i;
        r->in = p->fista_hat, r->in2 = p->yhat, r->out = p->rh, r->partials = p->red.partials;
        r = b->nurec[NK_ADJ_FISTA].host.data() + i;
        r->in = p->rh, r->in2 = nullptr, r->out = p->ghat, r->partials = nullptr;
        SumRec& sr = b->sumrec.host[i];
        sr.part_r = p->red.partials;
        sr.nr = rb;
        sr.part_f = p->red.partials + (size_t)rb * isam::kRedSlots;
        sr.nf = isam::lat_blocks(p, 0);
    }
    for (auto& r : b->latrec) r.valid = false;
    for (auto& r : b->nurec) r.valid = false;
    b->sumrec.valid = false;
}

const int2* map_of(isam_batch_t b, const Group& g, int which) { return b->maps + g.map_off[which]; }

// The scans' NUFFT constants as they are now (a scan's calibration may have changed through
// its own plan); the stop pointers of the solver records are kept.
void refresh_nu_args(isam_batch_t b) {
    for (int i = 0; i < b->n; ++i) {
        const isam::NufftArgs a = b->plans[i]->nufft_args();
        for (auto& r : b->nurec) {
            const int* stop = r.host[i].a.stop;
            r.host[i].a = a;
            r.host[i].a.stop = stop;
        }
    }
}



#define B_TRY(x)                                     \
    do {                                             \
        if ((x) != hipSuccess) return ISAM_EHIP;     \
    } while (0)

// One FISTA iteration over the whole batch (the captured sequence).
int iterate(isam_batch_t b, int norms, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, b->state);
    B_TRY(hipGetLastError());
    for (const Group& g : b->nu)
        B_TRY(isam::nufft_fwd_batch(g.key, b->nurec[NK_FWD_FISTA].dev, map_of(b, g, 0), g.nblk[0], s));
    for (const Group& g : b->nu)
        B_TRY(isam::nufft_adj_batch(g.key, b->nurec[NK_ADJ_FISTA].dev, map_of(b, g, 1), g.nblk[1], s));
    for (const Group& g : b->lat)
        B_TRY(isam::lat_fista_batch(g.key, g.sel_c, norms, b->latrec[LK_FISTA].dev, map_of(b, g, 0), g.nblk[0],
                                    &b->state->beta, s));
    if (norms) {
        hipLaunchKernelGGL(k_batch_stop, dim3(b->n), dim3(256), 0, s, b->sumrec.dev, b->stops, b->state);
        B_TRY(hipGetLastError());
    }
    return ISAM_OK;
}

void drop_graphs(isam_batch_t b) {
    for (auto& g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

int capture(isam_batch_t b, int norms) {
    if (b->graph[norms]) return ISAM_OK;
    hipGraph_t g = nullptr;
    B_TRY(hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed));
    const int rc = iterate(b, norms, b->cs);
    const hipError_t e = hipStreamEndCapture(b->cs, &g);
    if (rc != ISAM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != ISAM_OK ? rc : ISAM_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&b->graph[norms], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return ei == hipSuccess ? ISAM_OK : ISAM_EHIP;
}

void release(isam_batch_t b) {
    drop_graphs(b);
    for (isam_plan_t p : b->plans)
        if (p) isam_destroy(p);
    for (auto& r : b->latrec) r.release();
    for (auto& r : b->nurec) r.release();
    b->sumrec.release();
    void* dptr[] = {b->maps, b->stops, b->state, b->sums};
    for (void* q : dptr)
        if (q) (void)hipFree(q);
    if (b->host_stops) (void)hipHostFree(b->host_stops);
    if (b->host_sums) (void)hipHostFree(b->host_sums);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    for (hipStream_t q : b->ss)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

// Streams of the streams schedule: four, each with a hardware queue of its own.  Streams
// made by hipStreamCreate share the process's pool of hardware queues (four by default) with
// every other stream of the process, so two of them can land on one queue and then run one
// after the other (measured: 476 against 572 batch iterations/s on 64 uneven scans).  A
// stream with a CU mask gets a queue of its own; the mask names every CU of the device, so
// it restricts nothing.  Eight such streams ran slower than four (510).
constexpr int kSchedStreams = 4;

int ensure_streams(isam_batch_t b) {
    if (!b->ss.empty()) return ISAM_OK;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->plans[0]->device) != hipSuccess ||
        ncu < 1)
        return ISAM_EHIP;
    std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
    for (int c = 0; c < ncu; ++c) mask[c / 32] |= 1u << (c % 32);
    std::vector<hipStream_t> ss(kSchedStreams, nullptr);
    std::vector<hipEvent_t> ev(1, nullptr);      // the fork event
    int rc = ISAM_OK;
    for (auto& q : ss) {
        // a runtime that refuses the mask still gets a stream, from the shared queue pool
        if (rc == ISAM_OK && hipExtStreamCreateWithCUMask(&q, (uint32_t)mask.size(), mask.data()) != hipSuccess &&
            hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
            rc = ISAM_EHIP;
    }
    for (auto& e : ev)
        if (rc == ISAM_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = ISAM_EHIP;
    if (rc) {
        for (hipStream_t q : ss)
            if (q) (void)hipStreamDestroy(q);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        return rc;
    }
    b->ss = ss;
    b->ev = ev;
    b->order.resize(b->n);
    for (int i = 0; i < b->n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (int64_t)b->plans[x]->ncol * b->plans[x]->nk > (int64_t)b->plans[y]->ncol * b->plans[y]->nk;
    });
    return ISAM_OK;
}

// FISTA in the streams schedule: each scan's own solve (isam_fista_ex, so its result is that
// of isam_fista on the scan's plan, bit for bit) on one of the batch's streams, scans dealt to
// streams by decreasing size.  One host thread per stream enqueues its scans' solves one after
// another, each solve's host synchronisation holding up only its own stream.  The streams
// first wait for the caller's earlier work; every stream is complete on return.
int fista_streams(isam_batch_t b, const float* y, const float* lambda, const float* w, int max_iter, float tol,
                  const std::vector<double>& Ls, int add_residual, float2* out, isam_fista_info* info,
                  hipStream_t s) {
    int rc = ensure_streams(b);
    if (rc) return rc;
    const int ns = std::min((int)b->ss.size(), b->n);     // streams (and host threads) in use
    if (hipEventRecord(b->ev[0], s) != hipSuccess) return ISAM_EHIP;
    for (int k = 0; k < ns; ++k)
        if (hipStreamWaitEvent(b->ss[k], b->ev[0], 0) != hipSuccess) return ISAM_EHIP;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ISAM_EHIP;
    std::vector<int> st(b->n, ISAM_OK);
    std::vector<isam_fista_info> inf(b->n);
    auto worker = [&](int k) {
        const bool dev_ok = hipSetDevice(dev) == hipSuccess;
        for (int j = k; j < b->n; j += ns) {
            const int i = b->order[j];
            st[j] = dev_ok ? isam_fista_ex(b->plans[i], y + b->off[i], lambda[i], w ? w + b->off[i] : nullptr,
                                           max_iter, tol, Ls[i], add_residual, nullptr, nullptr, nullptr,
                                           out + b->off[i], &inf[j], b->ss[k])
                           : ISAM_EHIP;
        }
    };
    std::vector<std::thread> th;
    int spawned = 0;
    try {
        th.reserve(ns);
        for (; spawned < ns; ++spawned) th.emplace_back(worker, spawned);
    } catch (...) {
        // no thread for the remaining streams: their scans run on this thread
    }
    for (int k = spawned; k < ns; ++k) worker(k);
    for (auto& t : th) t.join();
    for (int k = 0; k < ns; ++k)
        if (hipStreamSynchronize(b->ss[k]) != hipSuccess) rc = ISAM_EHIP;
    std::vector<int> scan_status(b->n);
    for (int j = 0; j < b->n; ++j) {
        const int i = b->order[j];
        if (st[j] != ISAM_OK && st[j] != ISAM_ENONFINITE) rc = rc ? rc : st[j];
        scan_status[i] = st[j];
        if (info) info[i] = inf[j];
    }
    if (rc) return rc;
    for (int i = 0; i < b->n; ++i)
        if (scan_status[i] != ISAM_OK) return scan_status[i];
    return ISAM_OK;
}

bool overlaps(const void* a, size_t na, const void* c, size_t nc) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(c);
    return x < y + nc && y < x + na;
}

}  // namespace

extern "C" int isam_batch_plan(const isam_geometry* geoms, int nscans, void* stream, isam_batch_t* out) {
    if (!out) return ISAM_EINVAL;
    *out = nullptr;
    if (!geoms || nscans < 1) return ISAM_EINVAL;
    for (int i = 0; i < nscans; ++i)
        if (geoms[i].ny != 1) return ISAM_EUNSUPPORTED;        // batches hold B-scans
    isam_batch_s* b = new (std::nothrow) isam_batch_s();
    if (!b) return ISAM_ENOMEM;
    b->n = nscans;
    b->plans.assign(nscans, nullptr);
    b->off.assign(nscans + 1, 0);
    int rc = ISAM_OK;
    for (int i = 0; i < nscans && rc == ISAM_OK; ++i) {
        rc = isam_plan(&geoms[i], stream, &b->plans[i]);
        if (rc == ISAM_OK) b->off[i + 1] = b->off[i] + (int64_t)geoms[i].nx * geoms[i].nk;
    }
    if (rc != ISAM_OK) {
        release(b);
        return rc;
    }
    for (int i = 0; i < nscans; ++i) {
        isam_plan_s* p = b->plans[i];
        // the batch chooses the lateral tile widths per group (default, tuned or set); the
        // scans' own plans follow them, so that a scan and the batch compute alike
        p->lat_c = 0;
        p->lat_cr = 0;
        auto find = [](std::vector<Group>& gs, int key) -> Group& {
            for (Group& g : gs)
                if (g.key == key) return g;
            gs.push_back(Group{});
            gs.back().key = key;
            return gs.back();
        };
        find(b->nu, p->K).scans.push_back(i);
        find(b->lat, p->nx).scans.push_back(i);
    }
    for (auto& r : b->latrec) rc = rc ? rc : r.alloc(nscans);
    for (auto& r : b->nurec) rc = rc ? rc : r.alloc(nscans);
    rc = rc ? rc : b->sumrec.alloc(nscans);
    if (rc == ISAM_OK && hipMalloc((void**)&b->stops, nscans * sizeof(StopState)) != hipSuccess) rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipHostMalloc((void**)&b->host_stops, nscans * sizeof(StopState)) != hipSuccess)
        rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipMalloc((void**)&b->state, sizeof(BatchState)) != hipSuccess) rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipMalloc((void**)&b->sums, 2 * nscans * sizeof(double)) != hipSuccess) rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipHostMalloc((void**)&b->host_sums, 2 * nscans * sizeof(double)) != hipSuccess)
        rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) rc = ISAM_EHIP;
    if (rc == ISAM_OK) rc = build_maps(b);
    if (rc != ISAM_OK) {
        release(b);
        return rc;
    }
    fill_static_records(b);
    *out = b;
    return ISAM_OK;
}

extern "C" void isam_batch_destroy(isam_batch_t b) {
    if (b) release(b);
}

extern "C" int isam_batch_offsets(isam_batch_t b, int64_t* offsets) {
    if (!b || !offsets) return ISAM_EINVAL;
    for (int i = 0; i <= b->n; ++i) offsets[i] = b->off[i];
    return ISAM_OK;
}

extern "C" int isam_batch_scan_plan(isam_batch_t b, int i, isam_plan_t* out) {
    if (!b || !out || i < 0 || i >= b->n) return ISAM_EINVAL;
    *out = b->plans[i];
    return ISAM_OK;
}

extern "C" int isam_batch_set_calibration(isam_batch_t b, int i, double a2, double a3, double z_focus,
                                          void* stream) {
    if (!b || i < 0 || i >= b->n) return ISAM_EINVAL;
    const int rc = isam_set_calibration(b->plans[i], a2, a3, z_focus, stream);
    if (rc) return rc;
    const isam::NufftArgs a = b->plans[i]->nufft_args();
    for (auto& r : b->nurec) r.host[i].a = a, r.valid = false;
    return ISAM_OK;
}

extern "C" int isam_batch_forward(isam_batch_t b, const void* eta, float* s_out, void* stream) {
    if (!b || !eta || !s_out) return ISAM_EINVAL;
    const int64_t n = b->off[b->n];
    if (overlaps(eta, n * 8, s_out, n * 4)) return ISAM_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->n; ++i) {
        b->latrec[LK_C2C_FWD].host[i].in = static_cast<const float2*>(eta) + b->off[i];
        b->latrec[LK_C2R].host[i].out = s_out + b->off[i];
    }
    refresh_nu_args(b);
    int rc = b->latrec[LK_C2C_FWD].upload(s);
    rc = rc ? rc : b->latrec[LK_C2R].upload(s);
    rc = rc ? rc : b->nurec[NK_FWD_OP].upload(s);
    if (rc) return rc;
    for (const Group& g : b->lat)
        B_TRY(isam::lat_c2c_batch(g.key, g.sel_c, b->latrec[LK_C2C_FWD].dev, map_of(b, g, 0), g.nblk[0], -1, s));
    for (const Group& g : b->nu)
        B_TRY(isam::nufft_fwd_batch(g.key, b->nurec[NK_FWD_OP].dev, map_of(b, g, 0), g.nblk[0], s));
    for (const Group& g : b->lat)
        B_TRY(isam::lat_c2r_batch(g.key, g.sel_r, b->latrec[LK_C2R].dev, map_of(b, g, 1), g.nblk[1], s));
    return ISAM_OK;
}

extern "C" int isam_batch_adjoint(isam_batch_t b, const float* r, void* eta_out, void* stream) {
    if (!b || !r || !eta_out) return ISAM_EINVAL;
    const int64_t n = b->off[b->n];
    if (overlaps(r, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->n; ++i) {
        b->latrec[LK_R2C].host[i].in = r + b->off[i];
        b->latrec[LK_C2C_INV].host[i].out = static_cast<float2*>(eta_out) + b->off[i];
    }
    refresh_nu_args(b);
    int rc = b->latrec[LK_R2C].upload(s);
    rc = rc ? rc : b->latrec[LK_C2C_INV].upload(s);
    rc = rc ? rc : b->nurec[NK_ADJ_OP].upload(s);
    if (rc) return rc;
    for (const Group& g : b->lat)
        B_TRY(isam::lat_r2c_batch(g.key, g.sel_r, b->latrec[LK_R2C].dev, map_of(b, g, 1), g.nblk[1], s));
    for (const Group& g : b->nu)
        B_TRY(isam::nufft_adj_batch(g.key, b->nurec[NK_ADJ_OP].dev, map_of(b, g, 1), g.nblk[1], s));
    for (const Group& g : b->lat)
        B_TRY(isam::lat_c2c_batch(g.key, g.sel_c, b->latrec[LK_C2C_INV].dev, map_of(b, g, 0), g.nblk[0], +1, s));
    return ISAM_OK;
}

extern "C" int isam_batch_fista(isam_batch_t b, const float* y, const float* lambda, const float* w, int max_iter,
                                float tol, const double* L, int add_residual, int flags, void* eta_out,
                                isam_fista_info* info, void* stream) {
    if (!b || !y || !lambda || !eta_out || max_iter < 0 || !(tol >= 0.f)) return ISAM_EINVAL;
    const int64_t ntot = b->off[b->n];
    if (overlaps(y, ntot * 4, eta_out, ntot * 8)) return ISAM_EALIAS;
    if (w && overlaps(w, ntot * 4, eta_out, ntot * 8)) return ISAM_EALIAS;
    for (int i = 0; i < b->n; ++i)
        if (!(lambda[i] >= 0.f) || (L && !std::isfinite(L[i]))) return ISAM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int norms = tol > 0.f;
    std::vector<double> Ls(b->n);
    for (int i = 0; i < b->n; ++i) {
        Ls[i] = L ? L[i] : 0.0;
        if (Ls[i] <= 0) {
            const int rc = isam_lipschitz(b->plans[i], 50, 0, nullptr, &Ls[i], stream);
            if (rc) return rc;
        }
    }
    if (b->sched == ISAM_BATCH_SCHED_STREAMS)
        return fista_streams(b, y, lambda, w, max_iter, tol, Ls, add_residual, static_cast<float2*>(eta_out), info, s);
    refresh_nu_args(b);
    for (int i = 0; i < b->n; ++i) {
        isam_plan_s* p = b->plans[i];
        const int rc = isam::fista_prepare(p, y + b->off[i], w ? w + b->off[i] : nullptr, s);
        if (rc) return rc;
        LatScan& f = b->latrec[LK_FISTA].host[i];
        f.w = w ? p->wbuf : nullptr;
        f.fs.step = (float)(1.0 / Ls[i]);
        f.fs.lam = lambda[i];
        f.fs.beta = 0.f;
        f.fs.norms = norms;
        f.fs.stop = norms ? &b->stops[i].iter : nullptr;
        // without the Eq. 15 norms the adjoint writes the gradient step eta_hat - g_hat / L
        // and the update pass reads it in place of g_hat and eta_hat (as a single scan does)
        f.fs.pre = !norms && p->ny == 1;
        b->nurec[NK_FWD_FISTA].host[i].a.stop = norms ? &b->stops[i].iter : nullptr;
        isam::NufftArgs& aa = b->nurec[NK_ADJ_FISTA].host[i].a;
        aa.stop = norms ? &b->stops[i].iter : nullptr;
        aa.step_eta = f.fs.pre ? p->fista_hat : nullptr;
        aa.gstep = f.fs.step;
    }
    int rc = b->latrec[LK_FISTA].upload(s);
    rc = rc ? rc : b->nurec[NK_FWD_FISTA].upload(s);
    rc = rc ? rc : b->nurec[NK_ADJ_FISTA].upload(s);
    rc = rc ? rc : b->sumrec.upload(s);
    if (rc) return rc;
    const bool use_graph = !(flags & ISAM_BATCH_NO_GRAPH);
    if (use_graph && (rc = capture(b, norms))) return rc;
    hipLaunchKernelGGL(k_batch_reset, dim3((b->n + 255) / 256), dim3(256), 0, s, b->state, b->stops, b->n, tol);
    B_TRY(hipGetLastError());
    constexpr int kPoll = 16;
    bool stops_read = false;
    for (int k = 1; k <= max_iter; ++k) {
        if (use_graph) {
            B_TRY(hipGraphLaunch(b->graph[norms], s));
        } else if ((rc = iterate(b, norms, s))) {
            return rc;
        }
        if (norms && (k % kPoll == 0 || k == max_iter)) {
            B_TRY(hipMemcpyAsync(b->host_stops, b->stops, b->n * sizeof(StopState), hipMemcpyDeviceToHost, s));
            B_TRY(hipStreamSynchronize(s));
            stops_read = true;
            bool all = true;
            for (int i = 0; i < b->n; ++i) all = all && b->host_stops[i].iter != 0;
            if (all) break;
        }
    }
    if (max_iter > 0) {
        hipLaunchKernelGGL(k_batch_sums, dim3(b->n), dim3(256), 0, s, b->sumrec.dev, b->sums);
        B_TRY(hipGetLastError());
        B_TRY(hipMemcpyAsync(b->host_sums, b->sums, 2 * b->n * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    int status = ISAM_OK;
    for (int i = 0; i < b->n; ++i) {
        const int st = stops_read ? b->host_stops[i].status : ISAM_OK;
        rc = isam::fista_finish(b->plans[i], Ls[i], add_residual && st == ISAM_OK,
                                static_cast<float2*>(eta_out) + b->off[i], s);
        if (rc) return rc;
    }
    B_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < b->n; ++i) {
        int st = stops_read ? b->host_stops[i].status : ISAM_OK;
        const double resid2 = max_iter > 0 ? b->host_sums[2 * i] : 0.0;
        const double l1 = max_iter > 0 ? b->host_sums[2 * i + 1] : 0.0;
        if (!std::isfinite(resid2) || !std::isfinite(l1)) st = ISAM_ENONFINITE;
        if (st != ISAM_OK) status = st;
        if (info) {
            info[i].iters_run = stops_read && b->host_stops[i].iter ? b->host_stops[i].iter : max_iter;
            info[i].status = st;
            info[i].rel_res = stops_read ? b->host_stops[i].rel_res : -1.0;
            info[i].resid2 = resid2;
            info[i].l1 = l1;
            info[i].L = Ls[i];
        }
    }
    return status;
}

namespace {

// Times a short solve (zero data, 8 iterations; one call to warm up, then `reps` calls) in
// each FISTA schedule by the host clock, since every call synchronises and the streams
// schedule's host-side enqueueing is part of its cost, and keeps the faster schedule.
int tune_schedule(isam_batch_t b, int reps, hipStream_t s) {
    const int64_t ntot = b->off[b->n];
    float* y = nullptr;
    float2* out = nullptr;
    if (hipMalloc((void**)&y, ntot * sizeof(float)) != hipSuccess) return ISAM_ENOMEM;
    if (hipMalloc((void**)&out, ntot * sizeof(float2)) != hipSuccess) {
        (void)hipFree(y);
        return ISAM_ENOMEM;
    }
    int rc = hipMemsetAsync(y, 0, ntot * sizeof(float), s) == hipSuccess ? ISAM_OK : ISAM_EHIP;
    const std::vector<float> lam(b->n, 1.f);
    const std::vector<double> L(b->n, 1.0);
    constexpr int kIters = 8;
    double best = 1e300;
    int best_sched = b->sched;
    for (int sched : {ISAM_BATCH_SCHED_GROUPED, ISAM_BATCH_SCHED_STREAMS}) {
        if (rc) break;
        b->sched = sched;
        rc = isam_batch_fista(b, y, lam.data(), nullptr, kIters, 0.f, L.data(), 0, 0, out, nullptr, s);
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < reps && rc == ISAM_OK; ++r)
            rc = isam_batch_fista(b, y, lam.data(), nullptr, kIters, 0.f, L.data(), 0, 0, out, nullptr, s);
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc == ISAM_OK && dt < best) best = dt, best_sched = sched;
    }
    b->sched = best_sched;
    (void)hipFree(y);
    (void)hipFree(out);
    return rc;
}

}  // namespace

extern "C" int isam_batch_tune(isam_batch_t b, int reps, void* stream) {
    if (!b || reps < 1) return ISAM_EINVAL;
    // the timed passes reuse the scans' workspaces: earlier work on the caller's stream must be done
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return ISAM_EHIP;
    hipStream_t s = b->cs;
    // the timed passes run on the scans' own workspaces: clear them (no graph is being captured)
    for (isam_plan_t p : b->plans) {
        const size_t nb = (size_t)p->nx * p->nk * sizeof(float2);
        B_TRY(hipMemsetAsync(p->fista_hat, 0, nb, s));
        B_TRY(hipMemsetAsync(p->ghat, 0, nb, s));
        B_TRY(hipMemsetAsync(p->zblk, 0, nb, s));
        B_TRY(hipMemsetAsync(p->sbuf, 0, (size_t)p->nx * p->nk * sizeof(float), s));
    }
    hipLaunchKernelGGL(k_batch_reset, dim3((b->n + 255) / 256), dim3(256), 0, s, b->state, b->stops, b->n, 0.f);
    B_TRY(hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    B_TRY(hipEventCreate(&e0));
    B_TRY(hipEventCreate(&e1));
    int rc = ISAM_OK;
    // candidate tile widths; lateral lengths below 192 have one fixed width
    const int cands[] = {2, 4, 8};
    for (Group& g : b->lat) {
        if (g.key < 192) continue;
        for (int real = 0; real < 2 && rc == ISAM_OK; ++real) {
            float best = 1e30f;
            int best_sel = real ? g.sel_r : g.sel_c;
            for (int sel : cands) {
                (real ? g.sel_r : g.sel_c) = sel;
                if ((rc = build_maps(b))) break;
                fill_static_records(b);
                // time the group's pass on the scans' own workspaces (contents are scratch here)
                for (int i : g.scans) {
                    b->latrec[LK_R2C].host[i].in = b->plans[i]->sbuf;
                    b->latrec[LK_FISTA].host[i].fs = isam::FistaStep{0.f, 0.f, 0.f, 0, nullptr};
                    b->latrec[LK_FISTA].host[i].w = nullptr;
                }
                if ((rc = b->latrec[LK_R2C].upload(s)) || (rc = b->latrec[LK_FISTA].upload(s))) break;
                auto run = [&]() -> hipError_t {
                    return real ? isam::lat_r2c_batch(g.key, g.sel_r, b->latrec[LK_R2C].dev, map_of(b, g, 1),
                                                      g.nblk[1], s)
                                : isam::lat_fista_batch(g.key, g.sel_c, 0, b->latrec[LK_FISTA].dev, map_of(b, g, 0),
                                                        g.nblk[0], &b->state->beta, s);
                };
                if (run() != hipSuccess) { rc = ISAM_EHIP; break; }     // warm-up
                if (hipEventRecord(e0, s) != hipSuccess) { rc = ISAM_EHIP; break; }
                for (int r = 0; r < reps && rc == ISAM_OK; ++r)
                    if (run() != hipSuccess) rc = ISAM_EHIP;
                if (rc || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    rc = rc ? rc : ISAM_EHIP;
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) best = ms, best_sel = sel;
            }
            (real ? g.sel_r : g.sel_c) = best_sel;
        }
        for (int i : g.scans) {
            b->plans[i]->lat_c = g.sel_c;
            b->plans[i]->lat_cr = g.sel_r;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == ISAM_OK) rc = build_maps(b);
    fill_static_records(b);
    drop_graphs(b);
    if (hipStreamSynchronize(s) != hipSuccess && rc == ISAM_OK) rc = ISAM_EHIP;
    if (rc == ISAM_OK) rc = tune_schedule(b, reps, (hipStream_t)stream);
    return rc;
}

extern "C" int isam_batch_set_schedule(isam_batch_t b, int sched) {
    if (!b || (sched != ISAM_BATCH_SCHED_GROUPED && sched != ISAM_BATCH_SCHED_STREAMS)) return ISAM_EINVAL;
    b->sched = sched;
    return ISAM_OK;
}

extern "C" int isam_batch_schedule(isam_batch_t b, int* sched) {
    if (!b || !sched) return ISAM_EINVAL;
    *sched = b->sched;
    return ISAM_OK;
}

extern "C" int isam_batch_tiles(isam_batch_t b, int32_t* nx, int32_t* sel_c, int32_t* sel_r, int32_t cap,
                                int32_t* ngroups) {
    if (!b || !ngroups) return ISAM_EINVAL;
    *ngroups = (int32_t)b->lat.size();
    for (int i = 0; i < (int)b->lat.size() && i < cap; ++i) {
        if (nx) nx[i] = b->lat[i].key;
        if (sel_c) sel_c[i] = isam::lat_tile(b->lat[i].key, b->lat[i].sel_c, 0);
        if (sel_r) sel_r[i] = isam::lat_tile(b->lat[i].key, b->lat[i].sel_r, 1);
    }
    return ISAM_OK;
}

extern "C" int isam_batch_set_tiles(isam_batch_t b, int32_t nx, int32_t sel_c, int32_t sel_r) {
    if (!b) return ISAM_EINVAL;
    for (Group& g : b->lat)
        if (g.key == nx) {
            // the block maps are rewritten in place: no earlier work may still read them
            if (hipDeviceSynchronize() != hipSuccess) return ISAM_EHIP;
            g.sel_c = sel_c;
            g.sel_r = sel_r;
            for (int i : g.scans) {
                b->plans[i]->lat_c = sel_c;
                b->plans[i]->lat_cr = sel_r;
            }
            drop_graphs(b);
            const int rc = build_maps(b);
            fill_static_records(b);
            return rc;
        }
    return ISAM_EINVAL;
}
