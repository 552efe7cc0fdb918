// Lateral transforms of the ISAM operator: the unitary DFT over A-scans (F_<-> of
// Eq. 2, 16, 17), applied to every depth row / wavenumber column.
//
// Data are [nx][nk] with the column (depth or k) index contiguous, so the
// transform runs across rows at stride nk.  A workgroup owns a tile of C
// consecutive complex columns (2C real columns for the real transforms) over all
// nx rows: it reads C*8 contiguous bytes per row, transforms in LDS, writes back.
// Real data use the two-for-one trick: real columns (2c, 2c+1) travel as one
// complex lane, so a C2R/R2C pair costs what one complex transform costs.
//
// Kernels:
//   k_lat_c2c    complex <-> complex, sign -1 (F_<->) or +1 (F_<->^{-1})
//   k_lat_c2r    Hermitian half [nx/2+1][nk] -> real [nx][nk]   (Re of F^{-1}, Eq. 5)
//   k_lat_r2c    real [nx][nk] -> Hermitian half                (F of a real residual)
// Spectra (lateral-frequency side) and the FISTA state are column-blocked (blk); the
// object and spectra at the C ABI are row-major.
//   k_lat_fista  gradient step, soft threshold (Eq. 14), momentum (Alg. 1) and the
//                forward lateral transform of the next momentum point, with Eq. 15 norms
#pragma once
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "plan.hpp"

namespace isam {
namespace {

// Radix cap (log2) for a tile of C lanes of length N that should keep TT threads busy.
constexpr int lat_pick_l(int N, int C, int TT) {
    return (fft_length_ok(N, 4) && N * C / fft_radix(N, 0, 4) >= TT)   ? 4
           : (fft_length_ok(N, 3) && N * C / fft_radix(N, 0, 3) >= TT) ? 3
                                                                        : 2;
}

template <int N, int C_, int TT = 512>
struct LatCfg {
    static constexpr int C = C_;                             // complex lanes per tile
    static constexpr int L = lat_pick_l(N, C, TT);           // radix cap: keep TT threads busy
    static constexpr int RO = fft_radix(N, 0, L);
    static constexpr int NB = N / RO * C;
    static constexpr int T = NB < 64 ? 64 : (NB > TT ? TT : NB);
    static constexpr int SPAN = N / RO;
    // the tile, and at least room for the block-reduction scratch (4 values x 8 waves)
    static constexpr size_t LDS = (size_t)lds_size(N * C) * sizeof(float2) > 256 ? (size_t)lds_size(N * C) * sizeof(float2) : 256;
    using Fwd = LdsFft<N, C, T, -1, C, L>;
    using Inv = LdsFft<N, C, T, +1, C, L>;
    static_assert(Fwd::EPT == Inv::EPT, "layouts");
    static_assert(LDS <= 160 * 1024, "lateral tile exceeds the LDS of one CU");
    // The two-buffer form for tiles of 4096 points or more and at most 8 lanes, where two
    // fit in LDS: the x transforms of B-scans, whose few large tiles leave one workgroup per
    // CU anyway.  Smaller tiles, and the wide tiles of a volume's y transform, keep the LDS
    // that lets several workgroups share a CU.  Chained transforms skip the opening barrier
    // when the last pass reads the second buffer (odd pass count).  The transform of a
    // row-major input keeps one buffer (FX<false>): it measured slower with two.
    static constexpr bool TWO = N * C >= 4096 && C <= 8 && 2 * LDS <= 160 * 1024;
    template <bool USE>
    using FX = std::conditional_t<USE && TWO, LdsFft2<N, C, T, L>, LdsFft1<N, C, T, L>>;
    using F2 = FX<true>;
    static constexpr bool F2_OPEN = !TWO || F2::NP % 2 == 0;
    static constexpr size_t LDS2 = (size_t)F2::SIZE * sizeof(float2) > 256 ? (size_t)F2::SIZE * sizeof(float2) : 256;
    static_assert(F2::EPT == Fwd::EPT, "layouts");
    static_assert(LDS2 <= 160 * 1024, "two-buffer lateral tile exceeds the LDS of one CU");
};

// IB / OB: input / output in the column-blocked layout (else row-major [nx][nk]).
template <int N, int C, int SIGN, bool IB, bool OB>
ISAM_DEV void lat_c2c_body(const float2* in, float2* out, int nk, const float2* __restrict__ tw, float scale,
                           int tile, int ntiles) {
    using Cf = LatCfg<N, C>;
    using F = typename Cf::template FX<IB>;
    extern __shared__ float2 lds[];
    const int m0 = xcd_tile(tile, ntiles) * Cf::C;
    typename F::Tw twr;
    F::load(tw, threadIdx.x, twr);
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j)
                v[i * Cf::RO + j] = in[IB ? blk(b + j * Cf::SPAN, m0 + c, N) : (unsigned)(b + j * Cf::SPAN) * nk + m0 + c];
        }
    }
    F::template run<SIGN>(v, lds, twr, threadIdx.x, false);      // nothing has read lds yet
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j)
                out[OB ? blk(b + j * Cf::SPAN, m0 + c, N) : (unsigned)(b + j * Cf::SPAN) * nk + m0 + c] =
                    cscale(v[i * Cf::RO + j], scale);
        }
    }
}

template <int N, int C, int SIGN, bool IB, bool OB>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_c2c(const float2* in, float2* out, int nk,
                                                          const float2* __restrict__ tw, float scale,
                                                          unsigned slab_in, unsigned slab_out) {
    // grid.y: independent slabs (the y rows of a volume) at the given element strides
    lat_c2c_body<N, C, SIGN, IB, OB>(in + (size_t)blockIdx.y * slab_in, out + (size_t)blockIdx.y * slab_out, nk, tw,
                                     scale, blockIdx.x, gridDim.x);
}

// Batched: workgroup b runs tile map[b].y of scan map[b].x (all scans of one lateral length N).
template <int N, int C, int SIGN, bool IB, bool OB>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_c2c_batch(const LatScan* __restrict__ scans,
                                                                const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const LatScan& sc = scans[m.x];
    lat_c2c_body<N, C, SIGN, IB, OB>(static_cast<const float2*>(sc.in), static_cast<float2*>(sc.out), sc.nk,
                                     sc.tw, 1.0f / sqrtf((float)N), m.y, sc.ntiles);
}

// Two real columns (2c, 2c+1) of the C2R output as one complex lane: element x of the
// lane is Za[x] + i Zb[x], with Z[x] = conj(Z[N - x]) above N/2 (Z column-blocked).
template <int N>
ISAM_DEV float2 hermitian_pair(const float2* zh, int x, int col) {
    const int row = x <= N / 2 ? x : N - x;
    const float4 z = *reinterpret_cast<const float4*>(zh + blk(row, col, N / 2 + 1));
    return x <= N / 2 ? c2(z.x - z.w, z.y + z.z) : c2(z.x + z.w, z.z - z.y);
}

// Split the transform F of (ra + i rb) into the half spectra of ra and rb through LDS.
template <int N, int T, int C, int L>
ISAM_DEV void split_store(float2* lds, const float2 (&v)[LdsFft<N, C, T, -1, C, L>::EPT], float2* rh,
                          int /*nk*/, int n0, float scale) {
    using F = LdsFft<N, C, T, -1, C, L>;
    constexpr int RO = F::RO, SPAN = F::SPAN;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < RO; ++j) lds[lds_pad((b + j * SPAN) * C + c)] = v[i * RO + j];
        }
    }
    __syncthreads();
    const float h = 0.5f * scale;
    for (int o = threadIdx.x; o < (N / 2 + 1) * C; o += T) {
        const int l = o / C, c = o % C;
        const float2 A = lds[lds_pad(l * C + c)];
        const float2 B = cconj(lds[lds_pad((l == 0 ? 0 : N - l) * C + c)]);
        const float2 s = cadd(A, B), d = csub(A, B);
        *reinterpret_cast<float4*>(rh + blk(l, n0 + 2 * c, N / 2 + 1)) =
            make_float4(s.x * h, s.y * h, d.y * h, -d.x * h);
    }
}

template <int N, int C>
ISAM_DEV void lat_c2r_body(const float2* __restrict__ zh, float* __restrict__ s, int nk,
                           const float2* __restrict__ tw, float scale, int tile, int ntiles) {
    using Cf = LatCfg<N, C>;
    using F = typename Cf::F2;
    extern __shared__ float2 lds[];
    const int n0 = xcd_tile(tile, ntiles) * 2 * Cf::C;
    typename F::Tw twr;
    F::load(tw, threadIdx.x, twr);
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j)
                v[i * Cf::RO + j] = hermitian_pair<N>(zh, b + j * Cf::SPAN, n0 + 2 * c);
        }
    }
    F::template run<+1>(v, lds, twr, threadIdx.x, false);
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j)
                *reinterpret_cast<float2*>(s + (unsigned)(b + j * Cf::SPAN) * nk + n0 + 2 * c) =
                    cscale(v[i * Cf::RO + j], scale);
        }
    }
}

template <int N, int C>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_c2r(const float2* __restrict__ zh,
                                                          float* __restrict__ s, int nk,
                                                          const float2* __restrict__ tw, float scale,
                                                          unsigned slab_in, unsigned slab_out) {
    lat_c2r_body<N, C>(zh + (size_t)blockIdx.y * slab_in, s + (size_t)blockIdx.y * slab_out, nk, tw, scale, blockIdx.x,
                       gridDim.x);
}

template <int N, int C>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_c2r_batch(const LatScan* __restrict__ scans,
                                                                const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const LatScan& sc = scans[m.x];
    lat_c2r_body<N, C>(static_cast<const float2*>(sc.in), static_cast<float*>(sc.out), sc.nk, sc.tw,
                       1.0f / sqrtf((float)N), m.y, sc.ntiles);
}

template <int N, int C>
ISAM_DEV void lat_r2c_body(const float* __restrict__ r, float2* __restrict__ rh, int nk,
                           const float2* __restrict__ tw, float scale, int tile, int ntiles) {
    using Cf = LatCfg<N, C>;
    using F = typename Cf::F2;
    extern __shared__ float2 lds[];
    const int n0 = xcd_tile(tile, ntiles) * 2 * Cf::C;
    typename F::Tw twr;
    F::load(tw, threadIdx.x, twr);
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j)
                v[i * Cf::RO + j] =
                    *reinterpret_cast<const float2*>(r + (unsigned)(b + j * Cf::SPAN) * nk + n0 + 2 * c);
        }
    }
    F::template run<-1>(v, lds, twr, threadIdx.x, false);
    split_store<N, Cf::T, Cf::C, Cf::L>(lds, v, rh, nk, n0, scale);
}

template <int N, int C>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_r2c(const float* __restrict__ r,
                                                          float2* __restrict__ rh, int nk,
                                                          const float2* __restrict__ tw, float scale,
                                                          unsigned slab_in, unsigned slab_out) {
    lat_r2c_body<N, C>(r + (size_t)blockIdx.y * slab_in, rh + (size_t)blockIdx.y * slab_out, nk, tw, scale, blockIdx.x,
                       gridDim.x);
}

template <int N, int C>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_r2c_batch(const LatScan* __restrict__ scans,
                                                                const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const LatScan& sc = scans[m.x];
    lat_r2c_body<N, C>(static_cast<const float*>(sc.in), static_cast<float2*>(sc.out), sc.nk, sc.tw,
                       1.0f / sqrtf((float)N), m.y, sc.ntiles);
}

// Weighted complex soft threshold of Eq. 14 with threshold theta (theta = 0: identity).
// The hardware square root and reciprocal (about 1 ulp) replace the correctly rounded
// library forms, whose range scaling and division fix-ups cost more than the transform.
ISAM_DEV float2 soft_threshold(float2 u, float theta) {
    const float mag = __builtin_amdgcn_sqrtf(fmaf(u.x, u.x, u.y * u.y));
    const float sh = fmaxf(mag - theta, 0.f);
    const float f = theta > 0.f ? sh * __builtin_amdgcn_rcpf(sh + theta) : 1.f;
    return cscale(u, f);
}

template <int N, int C, bool NORMS>
ISAM_DEV void lat_fista_body(float2* __restrict__ eta_hat, const float2* __restrict__ ghat,
                             float2* __restrict__ z, const float* __restrict__ w, int /*nk: blocked*/,
                             const float2* __restrict__ tw, float scale, const FistaStep& fs,
                             float* __restrict__ partials, int tile, int ntiles) {
    using Cf = LatCfg<N, C>;
    using FI = typename Cf::F2;
    using FF = typename Cf::F2;
    constexpr int RO = Cf::RO, SPAN = Cf::SPAN;
    if (fs.stop && *fs.stop) return;                   // solver already stopped (uniform)
    extern __shared__ float2 lds[];
    const int m0 = xcd_tile(tile, ntiles) * Cf::C;
    // the twiddles of both transforms, fetched with the tile
    typename FI::Tw twr;
    FI::load(tw, threadIdx.x, twr);
    float2 v[FI::EPT];
    float2 gv[NORMS ? FI::EPT : 1];
#pragma unroll
    for (int i = 0; i < FI::BPTO; ++i) {
        int c, b;
        if (FI::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < RO; ++j) {
                const size_t off = blk(b + j * SPAN, m0 + c, N);
                // u_hat = eta_hat - step * g_hat, or as the adjoint already formed it
                if (!NORMS && fs.pre) {
                    v[i * RO + j] = ghat[off];
                } else {
                    v[i * RO + j] = grad_step(eta_hat[off], ghat[off], fs.step);
                    if constexpr (NORMS) gv[i * RO + j] = cscale(ghat[off], fs.step);
                }
            }
        }
    }
    // z^{k-1} (and w) are fetched before the inverse transform so their latency overlaps it
    float2 zpv[FI::EPT];
    float wv[FI::EPT];
#pragma unroll
    for (int i = 0; i < FI::BPTO; ++i) {
        int c, b;
        if (FI::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < RO; ++j) {
                const size_t off = blk(b + j * SPAN, m0 + c, N);
                zpv[i * RO + j] = z[off];
                wv[i * RO + j] = w ? w[off] : 1.f;
            }
        }
    }
    FI::template run<+1>(v, lds, twr, threadIdx.x, false);      // nothing has read lds yet
    if constexpr (NORMS) FI::template run<+1>(gv, lds, twr, threadIdx.x, Cf::F2_OPEN);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < FI::BPTO; ++i) {
        int c, b;
        if (FI::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < RO; ++j) {
                const size_t off = blk(b + j * SPAN, m0 + c, N);
                const float2 u = cscale(v[i * RO + j], scale);
                const float wt = wv[i * RO + j];
                const float2 zn = soft_threshold(u, fs.lam * fs.step * wt);
                const float2 zp = zpv[i * RO + j];
                z[off] = zn;
                if constexpr (NORMS) {
                    const float2 g = cscale(gv[i * RO + j], scale);
                    const float2 d = csub(zn, cadd(u, g));      // z - eta, eta = u + g
                    acc[0] += cabs2(d);
                    acc[1] += cabs2(g);
                    acc[2] += cabs2(csub(zn, u));               // z - eta + g
                }
                acc[3] += wt * __builtin_amdgcn_sqrtf(cabs2(zn));
                v[i * RO + j] = cadd(zn, cscale(csub(zn, zp), fs.beta));   // next momentum point
            }
        }
    }
    FF::template run<-1>(v, lds, twr, threadIdx.x, Cf::F2_OPEN);
#pragma unroll
    for (int i = 0; i < FF::BPTO; ++i) {
        int c, b;
        if (FF::outer(threadIdx.x, i, c, b)) {
#pragma unroll
            for (int j = 0; j < RO; ++j)
                eta_hat[blk(b + j * SPAN, m0 + c, N)] = cscale(v[i * RO + j], scale);
        }
    }
    __syncthreads();
    block_sum_store<Cf::T, 4>(acc, reinterpret_cast<float*>(lds), partials + tile * kRedSlots);
}

template <int N, int C, bool NORMS>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_fista(float2* __restrict__ eta_hat,
                                                            const float2* __restrict__ ghat,
                                                            float2* __restrict__ z,
                                                            const float* __restrict__ w, int nk,
                                                            const float2* __restrict__ tw, float scale,
                                                            FistaStep fs, float* __restrict__ partials,
                                                            unsigned slab) {
    const size_t o = (size_t)blockIdx.y * slab;
    lat_fista_body<N, C, NORMS>(eta_hat + o, ghat + o, z + o, w ? w + o : nullptr, nk, tw, scale, fs,
                                partials + (size_t)blockIdx.y * gridDim.x * kRedSlots, blockIdx.x, gridDim.x);
}

// Batched: the momentum weight of the iteration comes from the device (beta), the rest of
// the step from each scan's record.
template <int N, int C, bool NORMS>
__global__ __launch_bounds__((LatCfg<N, C>::T)) void k_lat_fista_batch(const LatScan* __restrict__ scans,
                                                                  const int2* __restrict__ map,
                                                                  const float* __restrict__ beta) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const LatScan& sc = scans[m.x];
    FistaStep fs = sc.fs;
    fs.beta = *beta;
    lat_fista_body<N, C, NORMS>(static_cast<float2*>(sc.out), static_cast<const float2*>(sc.in), sc.z, sc.w, sc.nk,
                                sc.tw, 1.0f / sqrtf((float)N), fs, sc.partials, m.y, sc.ntiles);
}

template <typename K>
void set_lds(K kern, size_t bytes) {
    set_max_lds((const void*)kern, bytes);
}

// sign -1: row-major object -> blocked lateral spectrum; sign +1: blocked -> row-major.
template <int N, int C>
hipError_t launch_c2c(const float2* in, float2* out, int nk, const float2* tw, int sign, hipStream_t s, int slabs,
                      unsigned slab_in, unsigned slab_out) {
    using Cf = LatCfg<N, C>;
    const float scale = 1.0f / sqrtf((float)N);
    const dim3 grid(nk / C, slabs);
    if (sign < 0) {
        set_lds(k_lat_c2c<N, C, -1, false, true>, Cf::LDS);
        ISAM_LAUNCH((k_lat_c2c<N, C, -1, false, true>), grid, dim3(Cf::T), Cf::LDS, s, in, out, nk, tw, scale,
                    slab_in, slab_out);
    } else {
        set_lds(k_lat_c2c<N, C, +1, true, false>, Cf::LDS2);
        ISAM_LAUNCH((k_lat_c2c<N, C, +1, true, false>), grid, dim3(Cf::T), Cf::LDS2, s, in, out, nk, tw, scale,
                    slab_in, slab_out);
    }
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_c2r(const float2* zh, float* sout, int nk, const float2* tw, hipStream_t s, int slabs,
                      unsigned slab_in, unsigned slab_out) {
    using Cf = LatCfg<N, C>;
    set_lds(k_lat_c2r<N, C>, Cf::LDS2);
    ISAM_LAUNCH((k_lat_c2r<N, C>), dim3(nk / (2 * C), slabs), dim3(Cf::T), Cf::LDS2, s, zh, sout, nk, tw,
                       1.0f / sqrtf((float)N), slab_in, slab_out);
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_r2c(const float* r, float2* rh, int nk, const float2* tw, hipStream_t s, int slabs,
                      unsigned slab_in, unsigned slab_out) {
    using Cf = LatCfg<N, C>;
    set_lds(k_lat_r2c<N, C>, Cf::LDS2);
    ISAM_LAUNCH((k_lat_r2c<N, C>), dim3(nk / (2 * C), slabs), dim3(Cf::T), Cf::LDS2, s, r, rh, nk, tw,
                       1.0f / sqrtf((float)N), slab_in, slab_out);
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_fista(float2* eh, const float2* gh, float2* z, const float* w, int nk, const float2* tw,
                        FistaStep fs, float* partials, hipStream_t s, int slabs, unsigned slab) {
    using Cf = LatCfg<N, C>;
    const dim3 grid(nk / C, slabs);
    const float scale = 1.0f / sqrtf((float)N);
    if (fs.norms) {
        set_lds(k_lat_fista<N, C, true>, Cf::LDS2);
        ISAM_LAUNCH((k_lat_fista<N, C, true>), grid, dim3(Cf::T), Cf::LDS2, s, eh, gh, z, w, nk, tw,
                           scale, fs, partials, slab);
    } else {
        set_lds(k_lat_fista<N, C, false>, Cf::LDS2);
        ISAM_LAUNCH((k_lat_fista<N, C, false>), grid, dim3(Cf::T), Cf::LDS2, s, eh, gh, z, w, nk, tw,
                           scale, fs, partials, slab);
    }
    return hipGetLastError();
}

// Batched launchers: nblk workgroups over the block map of one group of scans.  Plain
// launches (no timing events), so that they can be captured in a graph.
template <int N, int C>
hipError_t launch_c2c_batch(const LatScan* recs, const int2* map, int nblk, int sign, hipStream_t s) {
    using Cf = LatCfg<N, C>;
    if (sign < 0) {
        set_lds(k_lat_c2c_batch<N, C, -1, false, true>, Cf::LDS);
        hipLaunchKernelGGL((k_lat_c2c_batch<N, C, -1, false, true>), dim3(nblk), dim3(Cf::T), Cf::LDS, s, recs, map);
    } else {
        set_lds(k_lat_c2c_batch<N, C, +1, true, false>, Cf::LDS2);
        hipLaunchKernelGGL((k_lat_c2c_batch<N, C, +1, true, false>), dim3(nblk), dim3(Cf::T), Cf::LDS2, s, recs, map);
    }
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_c2r_batch(const LatScan* recs, const int2* map, int nblk, hipStream_t s) {
    using Cf = LatCfg<N, C>;
    set_lds(k_lat_c2r_batch<N, C>, Cf::LDS2);
    hipLaunchKernelGGL((k_lat_c2r_batch<N, C>), dim3(nblk), dim3(Cf::T), Cf::LDS2, s, recs, map);
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_r2c_batch(const LatScan* recs, const int2* map, int nblk, hipStream_t s) {
    using Cf = LatCfg<N, C>;
    set_lds(k_lat_r2c_batch<N, C>, Cf::LDS2);
    hipLaunchKernelGGL((k_lat_r2c_batch<N, C>), dim3(nblk), dim3(Cf::T), Cf::LDS2, s, recs, map);
    return hipGetLastError();
}

template <int N, int C>
hipError_t launch_fista_batch(int norms, const LatScan* recs, const int2* map, int nblk, const float* beta,
                              hipStream_t s) {
    using Cf = LatCfg<N, C>;
    if (norms) {
        set_lds(k_lat_fista_batch<N, C, true>, Cf::LDS2);
        hipLaunchKernelGGL((k_lat_fista_batch<N, C, true>), dim3(nblk), dim3(Cf::T), Cf::LDS2, s, recs, map, beta);
    } else {
        set_lds(k_lat_fista_batch<N, C, false>, Cf::LDS2);
        hipLaunchKernelGGL((k_lat_fista_batch<N, C, false>), dim3(nblk), dim3(Cf::T), Cf::LDS2, s, recs, map, beta);
    }
    return hipGetLastError();
}

}  // namespace

// Tile widths built per lateral length: C complex lanes per tile (2C real columns for the
// real transforms).  Small transforms use 8 lanes; from 256 A-scans up the plan picks one
// of {1, 2, 4, 8} (tunable).  The defaults, 8 lanes for complex passes and 4 for real ones,
// make a tile one 8-column block of the blocked layout: one contiguous run of memory.
#define ISAM_LAT_C(SEL, DEF, CALL)                                     \
    switch (SEL) {                                                     \
        case 1: { constexpr int C = 1; CALL; }                         \
        case 2: { constexpr int C = 2; CALL; }                         \
        case 8: { constexpr int C = N >= 2048 ? 4 : 8; CALL; }         \
        case 4: { constexpr int C = 4; CALL; }                         \
        default: { constexpr int C = DEF; CALL; }                      \
    }
#define ISAM_LAT_SWITCH(CALL) ISAM_LAT_DISPATCH(p->nx, p->lat_c, ISAM_LAT_DEF_C, CALL)
#define ISAM_LAT_SWITCH_R(CALL) ISAM_LAT_DISPATCH(p->nx, p->lat_cr, ISAM_LAT_DEF_CR, CALL)
// Default complex tile width: 8 lanes, but 4 above 1280 points, where an 8-lane tile of the
// update pass spills registers (1536 and 1792 points: 41.9 and 36.3 us against 18.3 and 19.0
// with 4 lanes, at 1024 depth columns) and 2048 points build no 8-lane tile.
#define ISAM_LAT_DEF_C (N > 1280 ? 4 : 8)
#define ISAM_LAT_DEF_CR 4
// Built lateral lengths: powers of two (up to 128 with fixed 8-lane tiles, above with a
// tunable width) and 3, 5, 7 times powers of two from 192 to 1792.
#define ISAM_LAT_S(NN, CALL) case NN: { constexpr int N = NN, C = 8; CALL; }
#define ISAM_LAT_L(NN, SEL, DEF, CALL) case NN: { constexpr int N = NN; ISAM_LAT_C(SEL, DEF, CALL) }
#define ISAM_LAT_DISPATCH(NXV, SEL, DEF, CALL)                                               \
    switch (NXV) {                                                                           \
        ISAM_LAT_S(1, CALL) ISAM_LAT_S(2, CALL) ISAM_LAT_S(4, CALL) ISAM_LAT_S(8, CALL)      \
        ISAM_LAT_S(16, CALL) ISAM_LAT_S(32, CALL) ISAM_LAT_S(64, CALL) ISAM_LAT_S(128, CALL) \
        ISAM_LAT_L(192, SEL, DEF, CALL) ISAM_LAT_L(256, SEL, DEF, CALL)                      \
        ISAM_LAT_L(320, SEL, DEF, CALL) ISAM_LAT_L(384, SEL, DEF, CALL)                      \
        ISAM_LAT_L(448, SEL, DEF, CALL) ISAM_LAT_L(512, SEL, DEF, CALL)                      \
        ISAM_LAT_L(640, SEL, DEF, CALL) ISAM_LAT_L(768, SEL, DEF, CALL)                      \
        ISAM_LAT_L(896, SEL, DEF, CALL) ISAM_LAT_L(1024, SEL, DEF, CALL)                     \
        ISAM_LAT_L(1280, SEL, DEF, CALL) ISAM_LAT_L(1536, SEL, DEF, CALL)                    \
        ISAM_LAT_L(1792, SEL, DEF, CALL) ISAM_LAT_L(2048, SEL, DEF, CALL)                    \
        default: return hipErrorInvalidValue;                                                \
    }

int lat_l_real(const isam_plan_s* p);   // radix cap (log2) of the real lateral FFT

}  // namespace isam
