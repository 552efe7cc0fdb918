// C entry points of the operator and of the MBIR solve (Eq. 12, Alg. 1).
//
// isam_forward   s = Re(K^ eta)             lateral FFT -> NUFFT pairs -> C2R
// isam_adjoint   eta = K^^H r               R2C -> transposed NUFFT pairs -> lateral IFFT
// isam_normal    A^H A eta                  lateral FFT -> NUFFT -> transposed NUFFT -> IFFT
// isam_fista     per iteration: NUFFT of the momentum point with the data subtracted in
//                lateral frequency -> transposed NUFFT -> update pass (IFFT, step, soft
//                threshold, momentum, FFT of the next momentum point).  The momentum point
//                is kept in lateral frequency, so an iteration is three passes.
#include <algorithm>
#include <cmath>
#include <limits>
#include <new>

#include "common.hpp"
#include "plan.hpp"

namespace isam {
thread_local PassEvents g_pass_events;
}

using namespace isam;

namespace {

// Maximum that keeps a NaN (fmax would drop it), so that a non-finite input reaches the host.
ISAM_DEV double nan_max(double a, double b) { return a != a ? a : (b != b ? b : fmax(a, b)); }
ISAM_DEV float nan_maxf(float a, float b) { return a != a ? a : (b != b ? b : fmaxf(a, b)); }

// FP64 sums (or maxima) of the per-workgroup partials: strided per-thread sums, then a
// fixed-order tree, so the result does not depend on scheduling.

ISAM_DEV void finalize_block(const float* __restrict__ partials, int nblocks, int nslots,
                             double* __restrict__ sums, int mode_max) {
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    for (int s = 0; s < nslots; ++s) {
        double acc = 0.0;
        for (int b = tid; b < nblocks; b += 256) {
            const double v = partials[b * kRedSlots + s];
            acc = mode_max ? nan_max(acc, v) : acc + v;
        }
        sh[tid] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) sh[tid] = mode_max ? nan_max(sh[tid], sh[tid + w]) : sh[tid] + sh[tid + w];
            __syncthreads();
        }
        if (tid == 0) sums[s] = sh[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_finalize(const float* __restrict__ partials, int nblocks,
                                                  int nslots, double* __restrict__ sums, int mode_max) {
    finalize_block(partials, nblocks, nslots, sums, mode_max);
}

// Two independent sums in one launch (block 0: a, block 1: b), as k_finalize.
__global__ __launch_bounds__(256) void k_finalize2(const float* __restrict__ pa, int na, int sa, double* __restrict__ da,
                                                   const float* __restrict__ pb, int nb, int sb,
                                                   double* __restrict__ db) {
    if (blockIdx.x == 0) finalize_block(pa, na, sa, da, 0);
    else finalize_block(pb, nb, sb, db, 0);
}

// Per-iteration record of the solve on the device (Eq. 15).  Sums slots 0..3 of the update
// pass's partials (||z - eta||^2, ||g||^2, ||z - eta + g||^2, sum w|z|) and slot 0 of the
// forward NUFFT's (||A eta - y||^2) in FP64 with a fixed-order tree and forms r_r.  With
// tol > 0 it records iteration k in st->iter once r_r < tol; a non-finite norm records k and
// the status ENONFINITE (so the solver kernels stop).  With hist, row `row` of hist receives
// (r_r, ||A eta^k - y||^2, sum w|z^k|).  Does nothing once a stop has been recorded.
__global__ __launch_bounds__(256) void k_stop_check(const float* __restrict__ part_f, int nf,
                                                    const float* __restrict__ part_r, int nr,
                                                    isam::StopState* st, int k, float tol,
                                                    double* __restrict__ hist, int row) {
    if (st->iter) return;                              // uniform
    __shared__ double sh[5][256];
    const int tid = threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < nf; b += 256)
        for (int i = 0; i < 4; ++i) acc[i] += part_f[b * kRedSlots + i];
    for (int b = tid; b < nr; b += 256) acc[4] += part_r[b * kRedSlots];
    for (int i = 0; i < 5; ++i) sh[i][tid] = acc[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int i = 0; i < 5; ++i) sh[i][tid] += sh[i][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const double d = sh[0][0], g = sh[1][0], e = sh[2][0], l1 = sh[3][0], r2 = sh[4][0];
        const double rr = sqrt(d) / (fmax(sqrt(g), sqrt(e)) + 1e-12);
        if (hist) {
            hist[3 * row] = rr;
            hist[3 * row + 1] = r2;
            hist[3 * row + 2] = l1;
        }
        if (!isfinite(d) || !isfinite(g) || !isfinite(e) || !isfinite(l1) || !isfinite(r2)) {
            st->status = ISAM_ENONFINITE;
            st->iter = k;
        } else {
            st->rel_res = rr;
            if (tol > 0.f && rr < (double)tol) st->iter = k;
        }
    }
}

// Partial sum of |x|^2 (slot 0) over a complex vector; 256 threads per block.
__global__ __launch_bounds__(256) void k_sumsq(const float2* __restrict__ x, size_t n,
                                               float* __restrict__ partials) {
    __shared__ float scratch[4];
    float acc[1] = {0.f};
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        acc[0] += cabs2(x[i]);
    block_sum_store<256, 1>(acc, scratch, partials + blockIdx.x * kRedSlots);
}

// Partial max of |x_i| / w_i (slot 0).
__global__ __launch_bounds__(256) void k_absmax(const float2* __restrict__ x, const float* __restrict__ w,
                                                size_t n, float* __restrict__ partials) {
    __shared__ float scratch[4];
    float m = 0.f;
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        float v = sqrtf(cabs2(x[i]));
        if (w) v /= w[i];
        m = nan_maxf(m, v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = nan_maxf(m, __shfl_xor(m, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[blockIdx.x * kRedSlots] = nan_maxf(nan_maxf(scratch[0], scratch[1]), nan_maxf(scratch[2], scratch[3]));
}

// x *= 1 / sqrt(sums[slot])
__global__ void k_scale_inv_sqrt(float2* __restrict__ x, size_t n, const double* __restrict__ sums, int slot) {
    const float f = (float)(1.0 / sqrt(sums[slot]));
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = cscale(x[i], f);
}

// x -= a * y
__global__ void k_axpy(float2* __restrict__ x, const float2* __restrict__ y, float a, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = csub(x[i], cscale(y[i], a));
}

// Row-major real [slabs][rows][cols] -> column-blocked per slab, and back for complex data.
__global__ void k_to_blk_f(const float* __restrict__ src, float* __restrict__ dst, int rows, int cols, int slabs) {
    const size_t m = (size_t)rows * cols, n = m * slabs;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t j = i % m;
        dst[i - j + blk((int)(j / cols), (int)(j % cols), rows)] = src[i];
    }
}
__global__ void k_from_blk_c(const float2* __restrict__ src, float2* __restrict__ dst, int rows, int cols,
                             int slabs) {
    const size_t m = (size_t)rows * cols, n = m * slabs;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t j = i % m;
        dst[i] = src[i - j + blk((int)(j / cols), (int)(j % cols), rows)];
    }
}

// First iteration of a fresh FISTA solve (Alg. 1 starts from eta^1 = z^0 = 0).  A eta^1 = 0,
// so the forward pass's residual spectrum is -F(y): workgroup b writes it for the rows of
// column pair b (the forward NUFFT's pairs), with that pass's ||r||^2 partial for the pair
// (Parseval weights as there: a partner pair with one stored row counts it twice).  All
// workgroups also clear the two state arrays (the momentum point and the iterate, 2 n4
// complex values each), which the first adjoint and update pass read.
__global__ __launch_bounds__(256) void k_fista_first(const isam::FwdPair* __restrict__ pairs, int nk, int nh,
                                                     const float2* __restrict__ yhat, float2* __restrict__ rh,
                                                     float* __restrict__ partials, float4* __restrict__ sa,
                                                     float4* __restrict__ sb, size_t n4) {
    __shared__ float red[4];
    const isam::FwdPair pr = pairs[blockIdx.x];
    float acc[1] = {0.f};
    for (int i = threadIdx.x; i < nk; i += 256) {
        const unsigned oa = blk(pr.ha, i, nh);
        const float2 a = yhat[oa];
        rh[oa] = c2(-a.x, -a.y);
        if (pr.hb >= 0) {
            const unsigned ob = blk(pr.hb, i, nh);
            const float2 b = yhat[ob];
            rh[ob] = c2(-b.x, -b.y);
            acc[0] += cabs2(a) + cabs2(b);
        } else {
            acc[0] += (pr.mode == 0 ? 2.f : 1.f) * cabs2(a);
        }
    }
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256) {
        sa[i] = z4;
        sb[i] = z4;
    }
    block_sum_store<256, 1>(acc, red, partials + blockIdx.x * kRedSlots);
}

// End of a FISTA solve in one launch.  Workgroups [0, nconv): z^k from the blocked layout
// into the row-major output.  Workgroup nconv: ||A eta^k - y||^2 from the forward pass's
// partials (pa, na workgroups, slot 0) into hsums[0].  Workgroup nconv + 1: the update pass's
// four sums (pb, nb workgroups, slots 0..3) into hsums[1..4], and the stop state into hstop
// if non-null.  hsums and hstop are device addresses of pinned host records.
__global__ __launch_bounds__(256) void k_fista_end(const float2* __restrict__ src, float2* __restrict__ dst,
                                                   int rows, int cols, int slabs, int nconv,
                                                   const float* __restrict__ pa, int na,
                                                   const float* __restrict__ pb, int nb, double* hsums,
                                                   const isam::StopState* __restrict__ st,
                                                   isam::StopState* hstop) {
    if ((int)blockIdx.x < nconv) {
        const size_t m = (size_t)rows * cols, n = m * slabs;
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)nconv * blockDim.x) {
            const size_t j = i % m;
            dst[i] = src[i - j + blk((int)(j / cols), (int)(j % cols), rows)];
        }
    } else if ((int)blockIdx.x == nconv) {
        finalize_block(pa, na, 1, hsums, 0);
    } else {
        finalize_block(pb, nb, 4, hsums + 1, 0);
        if (hstop && threadIdx.x == 0) *hstop = *st;
    }
}

__global__ void k_zero(float2* __restrict__ x, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = c2(0.f, 0.f);
}

// FISTA start (Alg. 1: eta^1 = z^0 = 0): zero both state arrays (unless zero is 0) and reset
// the device stop state, in one launch.
__global__ void k_fista_init(float2* __restrict__ a, float2* __restrict__ b, size_t n, int zero,
                             isam::StopState* st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = 0;
        st->status = ISAM_OK;
        st->rel_res = -1.0;
    }
    if (!zero) return;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        a[i] = c2(0.f, 0.f);
        b[i] = c2(0.f, 0.f);
    }
}

// Counter-based complex Gaussian start vector: SplitMix64 (Steele, Lea & Flood 2014)
// on (seed, index), then the Box-Muller transform; CN(0, 1) entries.
__device__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void k_randn(float2* __restrict__ x, size_t n, uint64_t seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed ^ (2 * i)), b = splitmix64(seed ^ (2 * i + 1));
        const double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double r = sqrt(-log(u1));            // sqrt(-2 ln u1) / sqrt(2)
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        x[i] = make_float2((float)(r * cs), (float)(r * sn));
    }
}

int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 2048); }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char *pa = (const char*)a, *pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

#define HIP_OK(x)                                    \
    do {                                             \
        if ((x) != hipSuccess) return ISAM_EHIP;     \
    } while (0)

int sum_to_host(isam_plan_t p, const float* partials, int nblocks, int nslots, int mode_max, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, nblocks, nslots, p->red.sums, mode_max);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(p->host_sums, p->red.sums, nslots * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return ISAM_OK;
}

// Per-pass timing: while isam_timing is enabled, each pass's kernel launch carries an event pair
// that the runtime stamps with the kernel's begin and end.
int tbegin(isam_plan_t p, int tag, hipStream_t s) {
    if (!p->timing_on) return -1;
    if (p->tev_used == p->tev_cap) {
        const int cap = std::max(256, 2 * p->tev_cap);
        hipEvent_t* ev = new (std::nothrow) hipEvent_t[2 * cap];
        int* tg = new (std::nothrow) int[cap];
        if (!ev || !tg) {
            delete[] ev;
            delete[] tg;
            return -1;
        }
        for (int i = 0; i < 2 * p->tev_cap; ++i) ev[i] = p->tev[i];
        for (int i = 0; i < p->tev_cap; ++i) tg[i] = p->ttag[i];
        for (int i = 2 * p->tev_cap; i < 2 * cap; ++i)
            if (hipEventCreate(&ev[i]) != hipSuccess) ev[i] = nullptr;
        delete[] p->tev;
        delete[] p->ttag;
        p->tev = ev;
        p->ttag = tg;
        p->tev_cap = cap;
    }
    const int i = p->tev_used;
    if (!p->tev[2 * i] || !p->tev[2 * i + 1]) return -1;
    p->tev_used++;
    p->ttag[i] = tag;
    p->tstream = s;
    isam::g_pass_events.start = p->tev[2 * i];
    isam::g_pass_events.stop = p->tev[2 * i + 1];
    return i;
}

void tend(isam_plan_t, int, hipStream_t) { isam::g_pass_events = isam::PassEvents{}; }

}  // namespace

// Sum the recorded pairs into the per-pass totals (the stream must have completed them).
void isam_timing_collect(isam_plan_t p) {
    for (int i = 0; i < p->tev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->tev[2 * i], p->tev[2 * i + 1]) == hipSuccess) {
            p->tms[p->ttag[i]] += ms;
            p->tcnt[p->ttag[i]] += 1;
        }
    }
    p->tev_used = 0;
}

namespace {

#define TIMED(tag, expr)                               \
    do {                                               \
        const int t_ = tbegin(p, tag, s);              \
        const hipError_t e_ = (expr);                  \
        tend(p, t_, s);                                \
        if (e_ != hipSuccess) return ISAM_EHIP;        \
    } while (0)

// Lateral transforms of the whole object: over x for a B-scan; over x then y for a volume
// (x per slab into the slab-blocked x spectrum xs, then y, Eq. 2 in two dimensions).
// Lateral spectra use the column index lx * ny + ly (see the column tables).
int lat_fwd(isam_plan_t p, const float2* in, float2* out, hipStream_t s) {
    if (p->ny == 1) {
        TIMED(0, lat_c2c(p, in, out, -1, s));
    } else {
        TIMED(0, lat_c2c(p, in, p->xs, -1, s));
        TIMED(7, lat_c2c_y(p, p->xs, out, p->nx * p->nk, -1, s));
    }
    return ISAM_OK;
}
int lat_inv(isam_plan_t p, const float2* in, float2* out, hipStream_t s) {
    if (p->ny == 1) {
        TIMED(5, lat_c2c(p, in, out, +1, s));
    } else {
        TIMED(7, lat_c2c_y(p, in, p->xs, p->nx * p->nk, +1, s));
        TIMED(5, lat_c2c(p, p->xs, out, +1, s));
    }
    return ISAM_OK;
}
// Hermitian half spectrum -> real spectra (Eq. 5), and real spectra -> half spectrum.
int lat_to_real(isam_plan_t p, const float2* zh, float* out, hipStream_t s) {
    if (p->ny == 1) {
        TIMED(2, lat_c2r(p, zh, out, s));
    } else {
        TIMED(7, lat_c2c_y(p, zh, p->xsh, p->nh * p->nk, +1, s));
        TIMED(2, lat_c2r(p, p->xsh, out, s));
    }
    return ISAM_OK;
}
int lat_from_real(isam_plan_t p, const float* r, float2* rh, hipStream_t s) {
    if (p->ny == 1) {
        TIMED(3, lat_r2c(p, r, rh, s));
    } else {
        TIMED(3, lat_r2c(p, r, p->xsh, s));
        TIMED(7, lat_c2c_y(p, p->xsh, rh, p->nh * p->nk, -1, s));
    }
    return ISAM_OK;
}

#define LAT_TRY(x)                  \
    do {                            \
        const int rc_ = (x);        \
        if (rc_) return rc_;        \
    } while (0)

int forward_impl(isam_plan_t p, const float2* eta, float* s_out, hipStream_t s) {
    LAT_TRY(lat_fwd(p, eta, p->etahat, s));
    TIMED(1, nufft_fwd(p, p->etahat, nullptr, p->zh, nullptr, s));
    LAT_TRY(lat_to_real(p, p->zh, s_out, s));
    return ISAM_OK;
}

int adjoint_impl(isam_plan_t p, const float* r, float2* eta_out, hipStream_t s) {
    LAT_TRY(lat_from_real(p, r, p->rh, s));
    TIMED(4, nufft_adj(p, p->rh, p->ghat, s));
    LAT_TRY(lat_inv(p, p->ghat, eta_out, s));
    return ISAM_OK;
}

// out = A^H (A eta - y) (eta, out row-major; yhat = F(y) as a blocked half spectrum, or null).
// The lateral transform of the residual is Z - yhat (see k_nufft_fwd), so the forward and
// adjoint NUFFT passes meet in the lateral-frequency domain.  ||A eta - y||^2 partials go to
// red.partials slot 0 (nufft_fwd_blocks workgroups).
int normal_impl(isam_plan_t p, const float2* eta, const float2* yhat, float2* out, hipStream_t s) {
    LAT_TRY(lat_fwd(p, eta, p->etahat, s));
    TIMED(1, nufft_fwd(p, p->etahat, yhat, p->rh, p->red.partials, s));
    TIMED(4, nufft_adj(p, p->rh, p->ghat, s));
    LAT_TRY(lat_inv(p, p->ghat, out, s));
    return ISAM_OK;
}

}  // namespace

extern "C" int isam_forward(isam_plan_t p, const void* eta, float* s_out, void* stream) {
    if (!p || !eta || !s_out) return ISAM_EINVAL;
    const size_t n = (size_t)p->ncol * p->nk;
    if (overlaps(eta, n * 8, s_out, n * 4)) return ISAM_EALIAS;
    return forward_impl(p, (const float2*)eta, s_out, (hipStream_t)stream);
}

extern "C" int isam_adjoint(isam_plan_t p, const float* r, void* eta_out, void* stream) {
    if (!p || !r || !eta_out) return ISAM_EINVAL;
    const size_t n = (size_t)p->ncol * p->nk;
    if (overlaps(r, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    return adjoint_impl(p, r, (float2*)eta_out, (hipStream_t)stream);
}

extern "C" int isam_normal(isam_plan_t p, const void* eta, void* eta_out, void* stream) {
    if (!p || !eta || !eta_out) return ISAM_EINVAL;
    const size_t n = (size_t)p->ncol * p->nk;
    if (overlaps(eta, n * 8, eta_out, n * 8)) return ISAM_EALIAS;
    return normal_impl(p, (const float2*)eta, nullptr, (float2*)eta_out, (hipStream_t)stream);
}

extern "C" int isam_lipschitz(isam_plan_t p, int iters, uint64_t seed, const void* x0, double* L_out,
                              void* stream) {
    if (!p || !L_out || iters < 1) return ISAM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)p->ncol * p->nk;
    float2* x = p->vec;
    if (x0) {
        HIP_OK(hipMemcpyAsync(x, x0, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(k_randn, dim3(grid_for(n)), dim3(256), 0, s, x, n, seed);
        HIP_OK(hipGetLastError());
    }
    const int gb = grid_for(n);
    const int rb = nufft_fwd_blocks(p);
    // normalise the start vector into red.sums[1]
    hipLaunchKernelGGL(k_sumsq, dim3(gb), dim3(256), 0, s, x, n, p->red.partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, p->red.partials, gb, 1, p->red.sums + 1, 0);
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(gb), dim3(256), 0, s, x, n, p->red.sums, 1);
    HIP_OK(hipGetLastError());
    for (int it = 0; it < iters; ++it) {
        // ||A x||^2 (the Rayleigh quotient, ||x|| = 1) lands in sums[0]; x <- A^H A x / ||.||
        int rc = normal_impl(p, x, nullptr, x, s);   // in-place lateral pass is safe (tile-local)
        if (rc) return rc;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, p->red.partials, rb, 1, p->red.sums, 0);
        hipLaunchKernelGGL(k_sumsq, dim3(gb), dim3(256), 0, s, x, n, p->red.partials);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, p->red.partials, gb, 1, p->red.sums + 1, 0);
        hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(gb), dim3(256), 0, s, x, n, p->red.sums, 1);
        HIP_OK(hipGetLastError());
    }
    HIP_OK(hipMemcpyAsync(p->host_sums, p->red.sums, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    isam_timing_collect(p);
    const double ray = p->host_sums[0];
    if (!std::isfinite(ray)) return ISAM_ENONFINITE;
    *L_out = 1.01 * ray;
    return ISAM_OK;
}

extern "C" int isam_lambda_max(isam_plan_t p, const float* y, const float* w, double* out, void* stream) {
    if (!p || !y || !out) return ISAM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)p->ncol * p->nk;
    int rc = adjoint_impl(p, y, p->vec, s);
    if (rc) return rc;
    const int gb = grid_for(n);
    hipLaunchKernelGGL(k_absmax, dim3(gb), dim3(256), 0, s, p->vec, w, n, p->red.partials);
    HIP_OK(hipGetLastError());
    rc = sum_to_host(p, p->red.partials, gb, 1, 1, s);
    if (rc) return rc;
    *out = p->host_sums[0];
    return std::isfinite(*out) ? ISAM_OK : ISAM_ENONFINITE;
}

extern "C" int isam_calibration_grad(isam_plan_t p, const void* eta, const float* g, double* grad_out,
                                     void* stream) {
    if (!p || !eta || !g || !grad_out) return ISAM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (int rc = lat_fwd(p, (const float2*)eta, p->etahat, s)) return rc;
    if (int rc = lat_from_real(p, g, p->rh, s)) return rc;
    if (nufft_calgrad(p, p->etahat, p->rh, p->red.partials, s) != hipSuccess) return ISAM_EHIP;
    const int rc = sum_to_host(p, p->red.partials, nufft_fwd_blocks(p), 3, 0, s);
    if (rc) return rc;
    for (int i = 0; i < 3; ++i) {
        grad_out[i] = p->host_sums[i];
        if (!std::isfinite(grad_out[i])) return ISAM_ENONFINITE;
    }
    return ISAM_OK;
}

namespace isam {

// FISTA set-up (Alg. 1 with eta^1 = z^0 = 0): zero the state, bring the weights into the
// blocked layout, and form the data's lateral spectrum yhat = F(y) (Hermitian half, blocked).
int fista_prepare(isam_plan_t p, const float* y, const float* w, hipStream_t s, bool zero_state) {
    const size_t n = (size_t)p->ncol * p->nk;
    const int gb = grid_for(n);
    if (nufft_fwd_blocks(p) + lat_blocks(p, 0) > p->red.maxBlocks) return ISAM_EUNSUPPORTED;
    hipLaunchKernelGGL(k_fista_init, dim3(zero_state ? gb : 1), dim3(256), 0, s, p->zblk, p->fista_hat, n,
                       zero_state ? 1 : 0, p->stop);
    if (w) hipLaunchKernelGGL(k_to_blk_f, dim3(gb), dim3(256), 0, s, w, p->wbuf, p->nx, p->nk, p->ny);
    HIP_OK(hipGetLastError());
    return lat_from_real(p, y, p->yhat, s);
}

// FISTA output: z^k in row-major order, plus the optional residual step of Alg. 1,
// z += (1/L) A^H (y - A z).
int fista_finish(isam_plan_t p, double L, int add_residual, float2* out, hipStream_t s, bool convert) {
    const size_t n = (size_t)p->ncol * p->nk;
    const int gb = grid_for(n);
    if (convert) {
        hipLaunchKernelGGL(k_from_blk_c, dim3(gb), dim3(256), 0, s, p->zblk, out, p->nx, p->nk, p->ny);
        HIP_OK(hipGetLastError());
    }
    if (add_residual) {
        int rc = normal_impl(p, out, p->yhat, p->vec, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_axpy, dim3(gb), dim3(256), 0, s, out, p->vec, (float)(1.0 / L), n);
        HIP_OK(hipGetLastError());
    }
    return ISAM_OK;
}

}  // namespace isam

extern "C" int isam_fista_state_bytes(isam_plan_t p, int64_t* bytes) {
    if (!p || !bytes) return ISAM_EINVAL;
    *bytes = (int64_t)2 * p->ncol * p->nk * (int64_t)sizeof(float2);
    return ISAM_OK;
}

extern "C" int isam_fista_ex(isam_plan_t p, const float* y, float lambda, const float* w, int max_iter,
                             float tol, double L, int add_residual, const isam_fista_state* resume,
                             isam_fista_state* save, double* history, void* eta_out, isam_fista_info* info,
                             void* stream) {
    if (!p || !y || !eta_out || max_iter < 0 || !(lambda >= 0.f) || !(tol >= 0.f) || !std::isfinite(L))
        return ISAM_EINVAL;
    if (resume && (!resume->data || resume->k < 0 || !(resume->t >= 1.0) || !std::isfinite(resume->t)))
        return ISAM_EINVAL;
    if (save && !save->data) return ISAM_EINVAL;
    const size_t n = (size_t)p->ncol * p->nk;
    if (overlaps(y, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    if (w && overlaps(w, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    if (save && (overlaps(save->data, 2 * n * 8, eta_out, n * 8) || overlaps(save->data, 2 * n * 8, y, n * 4) ||
                 (w && overlaps(save->data, 2 * n * 8, w, n * 4))))
        return ISAM_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    if (L <= 0) {
        const int rc = isam_lipschitz(p, 50, 0, nullptr, &L, stream);
        if (rc) return rc;
    }
    if (history && max_iter > p->hist_cap) {
        double* h = nullptr;
        if (hipStreamSynchronize(s) != hipSuccess) return ISAM_EHIP;
        if (hipMalloc((void**)&h, (size_t)max_iter * 3 * sizeof(double)) != hipSuccess) return ISAM_ENOMEM;
        if (p->hist) (void)hipFree(p->hist);
        p->hist = h;
        p->hist_cap = max_iter;
    }
    // A fresh solve starts from eta^1 = z^0 = 0 (Alg. 1).  Its first iteration replaces the
    // forward pass of that zero input by k_fista_first, which also clears the state arrays,
    // so they are cleared up front only when no iteration runs.
    const bool fresh = resume == nullptr;
    static_assert(sizeof(float4) == 2 * sizeof(float2), "state arrays cleared two values at a time");
    {
        const int rc = isam::fista_prepare(p, y, w, s, fresh && max_iter == 0);
        if (rc) return rc;
    }
    // resume: the momentum point (lateral spectrum) and the last iterate, as saved
    const int kbase = resume ? resume->k : 0;
    if (resume) {
        HIP_OK(hipMemcpyAsync(p->fista_hat, resume->data, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
        HIP_OK(hipMemcpyAsync(p->zblk, (const float2*)resume->data + n, n * sizeof(float2),
                              hipMemcpyDeviceToDevice, s));
    }
    float2* z = p->zblk;
    float* wb = w ? p->wbuf : nullptr;
    const int rb = nufft_fwd_blocks(p), fb = lat_blocks(p, 0);
    float* part_r = p->red.partials;                            // forward NUFFT, slot 0
    float* part_f = p->red.partials + (size_t)rb * kRedSlots;   // update pass, slots 0..3
    FistaStep fs;
    fs.step = (float)(1.0 / L);
    fs.lam = lambda;
    fs.norms = tol > 0.f || history != nullptr;
    // Without the Eq. 15 norms (which need g_hat itself) the adjoint of a B-scan writes the
    // gradient step eta_hat - g_hat / L, so the update pass reads one array instead of two.
    // (A volume's adjoint output still passes through its y transform first.)
    fs.pre = !fs.norms && p->ny == 1;
    // With the norms, Eq. 15 (and the history row) is evaluated on the device after every
    // update pass; once a stop holds, every later solver kernel returns at once, so the state
    // stays that of the stopping iteration.  With a tolerance the host reads the stop state
    // every kPoll iterations.
    constexpr int kPoll = 16;
    const int* stop = fs.norms ? &p->stop->iter : nullptr;
    fs.stop = stop;
    const bool vol = p->ny > 1;
    const double t_start = resume ? resume->t : 1.0;
    double t = t_start;
    bool polled_stop = false;
    for (int it = 1; it <= max_iter; ++it) {
        const int k = kbase + it;
        if (fresh && it == 1) {
            // eta^1 = 0: the residual spectrum is -F(y), and the state arrays are cleared here
            hipLaunchKernelGGL(k_fista_first, dim3(rb), dim3(256), 0, s, p->pairs, p->nk, p->nhalf, p->yhat,
                               p->rh, part_r, reinterpret_cast<float4*>(p->fista_hat),
                               reinterpret_cast<float4*>(p->zblk), n / 2);
            HIP_OK(hipGetLastError());
        } else {
            // the momentum point lives in the x spectrum; a volume's NUFFT needs the y transform too
            const float2* eh = p->fista_hat;
            if (vol) {
                TIMED(7, lat_c2c_y(p, p->fista_hat, p->etahat, p->nx * p->nk, -1, s));
                eh = p->etahat;
            }
            TIMED(1, nufft_fwd(p, eh, p->yhat, p->rh, part_r, s, stop));
        }
        TIMED(4, nufft_adj(p, p->rh, p->ghat, s, stop, fs.pre ? p->fista_hat : nullptr, fs.step));
        const float2* gx = p->ghat;
        if (vol) {
            TIMED(7, lat_c2c_y(p, p->ghat, p->xs, p->nx * p->nk, +1, s));
            gx = p->xs;
        }
        const double t_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        fs.beta = (float)((t - 1.0) / t_next);
        TIMED(6, lat_fista(p, p->fista_hat, gx, z, wb, fs, part_f, s));
        if (fs.norms) {
            hipLaunchKernelGGL(k_stop_check, dim3(1), dim3(256), 0, s, part_f, fb, part_r, rb, p->stop, k, tol,
                               history ? p->hist : nullptr, it - 1);
            HIP_OK(hipGetLastError());
            if (tol > 0.f && (it % kPoll == 0 || it == max_iter)) {
                HIP_OK(hipMemcpyAsync(p->host_stop, p->stop, sizeof(isam::StopState), hipMemcpyDeviceToHost, s));
                HIP_OK(hipStreamSynchronize(s));
                polled_stop = it == max_iter;
                if (p->host_stop->iter) {
                    polled_stop = true;
                    break;
                }
            }
        }
        t = t_next;
    }
    // One synchronisation at the end: the output, the final norms (||A eta^k - y||^2 from the
    // last forward pass, the update pass's four sums), the stop state, the saved state and the
    // history are all enqueued first.  One kernel writes the output and the norms and stop
    // state, the latter straight into the pinned host records.  Those are first set to NaN
    // (and a zero stop state), so that a record the kernel did not write cannot pass for a
    // result.
    if (max_iter > 0) {
        for (int i = 0; i < 5; ++i) p->host_sums[i] = std::numeric_limits<double>::quiet_NaN();
        if (fs.norms && !polled_stop) {
            p->host_stop->iter = 0;
            p->host_stop->status = ISAM_ENONFINITE;
            p->host_stop->rel_res = std::numeric_limits<double>::quiet_NaN();
        }
        const int cb = grid_for(n);
        hipLaunchKernelGGL(k_fista_end, dim3(cb + 2), dim3(256), 0, s, p->zblk, (float2*)eta_out, p->nx, p->nk,
                           p->ny, cb, part_r, rb, part_f, fb, p->host_sums_dev, p->stop,
                           fs.norms && !polled_stop ? p->host_stop_dev : nullptr);
        HIP_OK(hipGetLastError());
    }
    if (save) {
        HIP_OK(hipMemcpyAsync(save->data, p->fista_hat, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
        HIP_OK(hipMemcpyAsync((float2*)save->data + n, p->zblk, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    {
        // the output conversion is done above when iterations ran
        const int rc = isam::fista_finish(p, L, add_residual, (float2*)eta_out, s, max_iter == 0);
        if (rc) return rc;
    }
    HIP_OK(hipStreamSynchronize(s));
    isam_timing_collect(p);
    int iters_run = max_iter, status = ISAM_OK;
    double rel_res = -1.0, resid2 = 0.0, l1 = 0.0;
    if (fs.norms && max_iter > 0) {
        if (tol > 0.f) rel_res = p->host_stop->rel_res;
        if (p->host_stop->iter) iters_run = p->host_stop->iter - kbase;
        status = p->host_stop->status;
    }
    if (max_iter > 0) {
        resid2 = p->host_sums[0];
        l1 = p->host_sums[4];
        if (!std::isfinite(resid2) || !std::isfinite(l1)) status = ISAM_ENONFINITE;
    }
    if (history && iters_run > 0) HIP_OK(hipMemcpy(history, p->hist, (size_t)iters_run * 3 * sizeof(double),
                                                   hipMemcpyDeviceToHost));
    if (save) {
        double ts = t_start;
        for (int i = 0; i < iters_run; ++i) ts = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * ts * ts));
        save->k = kbase + iters_run;
        save->t = ts;
    }
    if (info) {
        info->iters_run = iters_run;
        info->status = status;
        info->rel_res = rel_res;
        info->resid2 = resid2;
        info->l1 = l1;
        info->L = L;
    }
    return status;
}

extern "C" int isam_fista(isam_plan_t p, const float* y, float lambda, const float* w, int max_iter,
                          float tol, double L, int add_residual, void* eta_out, isam_fista_info* info,
                          void* stream) {
    return isam_fista_ex(p, y, lambda, w, max_iter, tol, L, add_residual, nullptr, nullptr, nullptr, eta_out,
                         info, stream);
}

extern "C" int isam_plan_stolt(isam_plan_t p, int col, int32_t* fl_out, float* tau_out, void* stream) {
    if (!p || !fl_out || !tau_out || col < 0 || col >= p->ncol) return ISAM_EINVAL;
    return inspect_stolt(p, col, fl_out, tau_out, (hipStream_t)stream) == hipSuccess ? ISAM_OK : ISAM_EHIP;
}

extern "C" int isam_plan_weights(isam_plan_t p, const float* tau, int n, void* w_out, void* stream) {
    if (!p || !tau || !w_out || n < 0) return ISAM_EINVAL;
    if (n == 0) return ISAM_OK;
    return inspect_weights(p, tau, n, (float2*)w_out, (hipStream_t)stream) == hipSuccess ? ISAM_OK : ISAM_EHIP;
}

extern "C" int isam_direct(isam_plan_t p, const float* y, void* eta_out, void* stream) {
    if (!p || !y || !eta_out) return ISAM_EINVAL;
    const size_t n = (size_t)p->ncol * p->nk;
    if (overlaps(y, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    const int t_ = tbegin(p, 8, s);
    const hipError_t e = direct_image(p, y, (float2*)eta_out, s);
    tend(p, t_, s);
    return e == hipSuccess ? ISAM_OK : ISAM_EHIP;
}

extern "C" int isam_timing(isam_plan_t p, int enable, double* ms_out, int64_t* count_out) {
    if (!p) return ISAM_EINVAL;
    if (p->tev_used > 0) {
        if (hipStreamSynchronize(p->tstream) != hipSuccess) return ISAM_EHIP;
        isam_timing_collect(p);
    }
    if (ms_out)
        for (int i = 0; i < ISAM_NPASS; ++i) ms_out[i] = p->tms[i];
    if (count_out)
        for (int i = 0; i < ISAM_NPASS; ++i) count_out[i] = p->tcnt[i];
    if (enable && !p->timing_on)
        for (int i = 0; i < ISAM_NPASS; ++i) {
            p->tms[i] = 0.0;
            p->tcnt[i] = 0;
        }
    p->timing_on = enable ? 1 : 0;
    return ISAM_OK;
}
