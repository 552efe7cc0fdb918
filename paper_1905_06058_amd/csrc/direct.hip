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
