// The "direct IFFT" image of Eq. 9 (Sec. "Methods under test"): each measured A-scan is
// dispersion-compensated by e^{-j phi(k)} and transformed along the spectral axis,
//   eta_d[p][m] = nk^{-1/2} sum_n y[p][n] e^{-j phi(k_n)} e^{-2 j k_n z_m},
// on the operator's full-range depth grid (row m in [-nk/2, nk/2) at index m + nk/2).
// With k_n = kc + (n - nk/2) dk and 2 dk dz = 2 pi / nk the kernel factors as
//   e^{-2 j k_n z_m} = e^{-2 j kc dz m} (-1)^m e^{-2 pi j n m / nk},
// so each A-scan is one nk-point forward FFT (in LDS) between two pointwise products:
// D_n = e^{-j phi(k_n)} before it and P_m = e^{-2 j kc dz m} (-1)^m / sqrt(nk) after it
// (both tables FP64-built, FP32-stored).  By Eq. 9 the result holds half of the object plus
// the doubly dispersed conjugate mirror; no lateral coupling, Stolt map, beam or focus.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "fft.hpp"
#include "plan.hpp"

namespace isam {
namespace {

template <int N>
struct DirCfg {
    static constexpr int RO = fft_radix(N, 0);
    static constexpr int NB = N / RO;
    static constexpr int T = NB < 64 ? 64 : (NB > 256 ? 256 : NB);
    using F = LdsFft<N, 1, T, -1>;
};

// One A-scan per workgroup: real samples in (coalesced: lane b reads x = b + j N/RO), the
// FFT in LDS, complex rows out at index (x + N/2) mod N.
template <int N>
__global__ __launch_bounds__(DirCfg<N>::T) void k_direct(const float* __restrict__ y, float2* __restrict__ out,
                                                         const float2* __restrict__ Dn,
                                                         const float2* __restrict__ Pm,
                                                         const float2* __restrict__ tw) {
    using Cf = DirCfg<N>;
    using F = typename Cf::F;
    __shared__ float2 lds[F::SIZE];
    const int tid = threadIdx.x;
    const size_t row = (size_t)blockIdx.x * N;
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(tid, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * F::SPAN;
                v[i * Cf::RO + j] = cscale(Dn[x], y[row + x]);
            }
        }
    }
    F::run(v, lds, tw, tid);
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(tid, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * F::SPAN;
                const int idx = (x + N / 2) & (N - 1);          // row m = x or x - N
                out[row + idx] = cmul(v[i * Cf::RO + j], Pm[idx]);
            }
        }
    }
}

// rows A-scans of nk samples, tables Dn, Pm and the staged nk-point twiddles tw
hipError_t launch_direct(int nk, int rows, const float* y, float2* out, const float2* Dn, const float2* Pm,
                         const float2* tw, hipStream_t s) {
#define ISAM_DIRECT_CASE(NN)                                                                  \
    case NN:                                                                                  \
        ISAM_LAUNCH(k_direct<NN>, dim3(rows), dim3(DirCfg<NN>::T), 0, s, y, out, Dn, Pm, tw); \
        return hipGetLastError();
    switch (nk) {
        ISAM_DIRECT_CASE(16)
        ISAM_DIRECT_CASE(32)
        ISAM_DIRECT_CASE(64)
        ISAM_DIRECT_CASE(128)
        ISAM_DIRECT_CASE(256)
        ISAM_DIRECT_CASE(512)
        ISAM_DIRECT_CASE(1024)
        ISAM_DIRECT_CASE(2048)
        ISAM_DIRECT_CASE(4096)
        default: return hipErrorInvalidValue;
    }
#undef ISAM_DIRECT_CASE
}

}  // namespace

hipError_t direct_image(const isam_plan_s* p, const float* y, float2* out, hipStream_t s) {
    return launch_direct(p->nk, p->ncol, y, out, p->Dn, p->Pm, p->twN, s);
}

}  // namespace isam

// ---------------------------------------------------------------------------------------
// The direct image without a plan and without allocating (isam_direct_static).  Its tables
// (Dn, Pm and the staged twiddles of the nk-point FFT: at most 2 * 4096 + 4352 complex
// entries, 100 KB) live in one file-scope device array.  Host code never passes the array's
// name to a kernel: the device address is looked up once per device with
// hipGetSymbolAddress and kept.
constexpr int kDirectMaxNk = 4096;
constexpr int kScratchEntries = 2 * kDirectMaxNk + isam::fft_stage_len(kDirectMaxNk, 4);
static __device__ __align__(256) float2 scratch[kScratchEntries];

namespace {

using namespace isam;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float2* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call on a device).
int scratch_address(float2** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ISAM_ENODEV;
    if (dev < 0 || dev >= kMaxDevices) return ISAM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ISAM_EHIP;
        g_scratch_ptr[dev] = static_cast<float2*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return ISAM_OK;
}

// Direct-image tables into the scratch array: Dn at [0, nk), Pm at [nk, 2 nk), the staged
// twiddles (exp(-2 pi i e / period), as the plan's table) at [2 nk, 2 nk + twlen).
__global__ void k_direct_tables(float2* __restrict__ tab, int nk, int twlen, double kc, double dk, double dz,
                                double a2, double a3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nk) direct_table_entry(i, nk, kc, dk, dz, a2, a3, tab[i], tab[nk + i]);
    if (i < twlen) {
        int e, period;
        fft_stage_entry(nk, 4, i, e, period);
        double sn, cs;
        sincospi(-2.0 * e / period, &sn, &cs);
        tab[2 * nk + i] = make_float2((float)cs, (float)sn);
    }
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char *pa = (const char*)a, *pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" int isam_direct_static(const isam_geometry* g, const float* y, void* eta_out, void* stream) {
    if (!g || !y || !eta_out) return ISAM_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->nk < 16) return ISAM_EINVAL;
    if (!std::isfinite(g->lambda_c) || !std::isfinite(g->dlambda) || !std::isfinite(g->a2) ||
        !std::isfinite(g->a3) || !(g->lambda_c > 0) || !(g->dlambda > 0) || !(g->dlambda < g->lambda_c))
        return ISAM_EINVAL;
    if ((g->nk & (g->nk - 1)) || g->nk > kDirectMaxNk) return ISAM_EUNSUPPORTED;   // beyond the scratch array
    const size_t rows = (size_t)g->nx * g->ny;
    if (rows > (size_t)1 << 30 || rows * g->nk > (size_t)1 << 30) return ISAM_EUNSUPPORTED;
    const size_t n = rows * g->nk;
    if (ranges_overlap(y, n * 4, eta_out, n * 8)) return ISAM_EALIAS;
    float2* tab = nullptr;
    if (int rc = scratch_address(&tab)) return rc;
    constexpr double kPi = 3.14159265358979323846;
    const double kc = 2.0 * kPi / g->lambda_c;
    const double band = 2.0 * kPi * g->dlambda / (g->lambda_c * g->lambda_c);
    const double dk = band / g->nk, dz = kPi / band;
    const int twlen = fft_stage_len(g->nk, 4);
    hipStream_t s = (hipStream_t)stream;
    const int nt = g->nk > twlen ? g->nk : twlen;
    hipLaunchKernelGGL(k_direct_tables, dim3((nt + 255) / 256), dim3(256), 0, s, tab, g->nk, twlen, kc, dk, dz,
                       g->a2, g->a3);
    if (hipGetLastError() != hipSuccess) return ISAM_EHIP;
    const hipError_t e = launch_direct(g->nk, (int)rows, y, (float2*)eta_out, tab, tab + g->nk, tab + 2 * g->nk, s);
    return e == hipSuccess ? ISAM_OK : ISAM_EHIP;
}
