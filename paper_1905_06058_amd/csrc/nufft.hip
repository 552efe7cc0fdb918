// Stolt resampling of the ISAM operator (Eq. 3, 16, 17) as a min-max NUFFT per
// lateral-frequency column.
//
// Forward, column l (eta_hat[l][m] given, m in [-nz/2, nz/2)):
//   Y[g]  = sum_m s_m eta_hat[l][m] exp(2 pi i g (m - mi) / K)     K = 2 nz, LDS FFT
//   X[n]  = B_l E_n f_n sum_j u~_j(tau_n) Y[(g0_n + j) mod K]       J = 6 taps from LDS
// with t_n = kz(l, n) dz K / (2 pi) in FP64, g0 = floor(t) - J/2, tau = t - floor(t),
// E_n = e^{i phi(k_n)} e^{2 i k_n z_f} / sqrt(nz), mi the integer part of the focal
// row, f_n = exp(-2 pi i m_r t_n / K) for its fractional part m_r, and u~ the min-max
// weights times exp(-2 pi i mi (tau + J/2 - j) / K).  Altogether this is
// c[l][n] X_N[l][n] with c = B e^{i phi} e^{i (2k - kz) z_f}: the integer focal
// shift moves into the FFT input placement, the rest into a per-n table and the weights.
//
// A workgroup takes the lateral pair (l, nx - l) (workgroup 0: the self-paired l = 0 and
// l = nx/2) and writes the Hermitian half Z[l] = (X[l] + conj X[nx - l]) / 2, which the
// C2R lateral pass turns into Re(F^{-1} X) (Eq. 5).
//
// Adjoint: the exact transpose.  The interpolation transpose is a gather: for each
// oversampled cell the contributing (n, j) are found from a per-column map, built in
// LDS, of the first sample reaching each unwrapped cell; t_n increases with n by at
// least 2 per sample, so each cell has about J/2 contributors and no atomics are needed.
#include <algorithm>

#include "common.hpp"
#include "fft.hpp"
#include "plan.hpp"

namespace isam {
namespace {

constexpr int kGsentinel = -(1 << 30);

template <int K>
struct NuCfg {
    static constexpr int NK = K / 2;
    static constexpr int P = ilog2(K);
    static constexpr int RO = 1 << fft_radix_log(P, 0);
    static constexpr int NB = K / RO;
    static constexpr int T = NB < 64 ? 64 : (NB > 256 ? 256 : NB);
    static constexpr int NPT = (NK + T - 1) / T;           // output samples per thread
    static constexpr int SPAN = K / RO;
    static constexpr int LOMAX = 2 * K;                    // unwrapped cells of one column
    using Fwd = LdsFft<K, 1, T, +1>;
    using Adj = LdsFft<K, 1, T, -1>;
    static constexpr size_t LDS_FWD = (size_t)(K + kWtabEntries) * sizeof(float2);
    static constexpr size_t AUX = (size_t)NK * (sizeof(float2) + sizeof(int) + sizeof(float)) +
                                  (size_t)LOMAX * sizeof(unsigned short);
    static constexpr size_t REGION = AUX > K * sizeof(float2) ? AUX : K * sizeof(float2);
    static constexpr size_t LDS_ADJ = (size_t)kWtabEntries * sizeof(float2) + REGION;
};

// Stolt grid position of sample n of a column with q^2 = q2 (FP64).  Returns false on an
// evanescent sample (4 k^2 <= q^2).  t = kz dz K / (2 pi); fl = floor(t); tau = t - fl.
ISAM_DEV bool stolt_point(const NufftArgs& a, double q2, int n, double& t, int& fl, float& tau) {
    const double k = a.kc + (double)(n - a.nk / 2) * a.dk;
    const double tk = 2.0 * k;
    const double d = fma(tk, tk, -q2);
    if (!(d > 0.0)) return false;
    t = sqrt(d) * a.cT;
    const double f = floor(t);
    fl = (int)f;
    tau = (float)(t - f);
    return true;
}

// Min-max weight of tap jj (0-based) at tau from the piecewise-cubic table in LDS.
ISAM_DEV float2 weight(const float2* wt, float tau, int jj) {
    const float tp = tau * kPieces;
    const int p = min((int)tp, kPieces - 1);
    const float x = tp - (float)p;
    const float4* row = reinterpret_cast<const float4*>(wt + (p * kJ + jj) * 4);
    const float4 a = row[0], b = row[1];     // (c0, c1), (c2, c3)
    float2 w;
    w.x = fmaf(fmaf(fmaf(b.z, x, b.x), x, a.z), x, a.x);
    w.y = fmaf(fmaf(fmaf(b.w, x, b.y), x, a.w), x, a.y);
    return w;
}

// The per-sample modulation B_l E_n f_n (f_n only with a fractional focal row).
ISAM_DEV float2 modulation(const NufftArgs& a, float Bl, int n, double t) {
    float2 e = cscale(a.En[n], Bl);
    if (a.has_frac) {
        double ph = a.mr_over_K * t;
        ph -= rint(ph);
        float s, c;
        sincospif(-2.0f * (float)ph, &s, &c);
        e = cmul(e, c2(c, s));
    }
    return e;
}

template <int K>
ISAM_DEV void forward_column(const NufftArgs& a, const float2* __restrict__ src, int col, float2* buf,
                             const float2* wt, float2 (&xt)[NuCfg<K>::NPT]) {
    using Cf = NuCfg<K>;
    using F = typename Cf::Fwd;
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * Cf::SPAN;
                const int u = (x + a.mi + a.nk / 2) & (K - 1);      // depth index placed at x
                v[i * Cf::RO + j] = u < a.nk ? cscale(src[u], a.sm[u]) : c2(0.f, 0.f);
            }
        }
    }
    F::run(v, buf, a.tw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) buf[b + j * Cf::SPAN] = v[i * Cf::RO + j];
        }
    }
    __syncthreads();
    const double q2 = a.q2[col];
    const float Bl = a.Bl[col];
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = threadIdx.x + r * Cf::T;
        float2 out = c2(0.f, 0.f);
        double t;
        int fl;
        float tau;
        if (n < a.nk && stolt_point(a, q2, n, t, fl, tau)) {
            const int base = fl - kJ / 2 + 1;                       // tap j = 1 at g0 + 1
            float2 acc = c2(0.f, 0.f);
#pragma unroll
            for (int jj = 0; jj < kJ; ++jj)
                acc = cfma(weight(wt, tau, jj), buf[(base + jj) & (K - 1)], acc);
            out = cmul(acc, modulation(a, Bl, n, t));
        }
        xt[r] = out;
    }
}

template <int K>
__global__ __launch_bounds__(NuCfg<K>::T) void k_nufft_fwd(const float2* __restrict__ etahat,
                                                           float2* __restrict__ zh, NufftArgs a) {
    using Cf = NuCfg<K>;
    extern __shared__ float2 smem[];
    float2* buf = smem;
    float2* wt = smem + K;
    for (int i = threadIdx.x; i < kWtabEntries; i += Cf::T) wt[i] = a.wtab[i];
    const int b = blockIdx.x;
    const int colA = b == 0 ? 0 : b;
    const int colB = b == 0 ? (a.nx >= 2 ? a.nx / 2 : -1) : a.nx - b;
    float2 xa[Cf::NPT], xb[Cf::NPT];
    forward_column<K>(a, etahat + (size_t)colA * a.nk, colA, buf, wt, xa);
    if (colB >= 0) forward_column<K>(a, etahat + (size_t)colB * a.nk, colB, buf, wt, xb);
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = threadIdx.x + r * Cf::T;
        if (n >= a.nk) continue;
        if (b == 0) {
            zh[n] = c2(xa[r].x, 0.f);
            if (colB >= 0) zh[(size_t)colB * a.nk + n] = c2(xb[r].x, 0.f);
        } else {
            zh[(size_t)b * a.nk + n] = cscale(cadd(xa[r], cconj(xb[r])), 0.5f);
        }
    }
}

template <int K>
ISAM_DEV void adjoint_column(const NufftArgs& a, const float2* __restrict__ rh, int rrow, bool conj_in,
                             int col, float2* region, const float2* wt, float2* __restrict__ dst,
                             int* s_nev) {
    using Cf = NuCfg<K>;
    using F = typename Cf::Adj;
    float2* V = region;
    int* G = reinterpret_cast<int*>(V + Cf::NK);
    float* TAU = reinterpret_cast<float*>(G + Cf::NK);
    unsigned short* LO = reinterpret_cast<unsigned short*>(TAU + Cf::NK);
    if (threadIdx.x == 0) *s_nev = a.nk;
    __syncthreads();
    const double q2 = a.q2[col];
    const float Bl = a.Bl[col];
    // phase A: Stolt points and modulated residual of every sample
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = threadIdx.x + r * Cf::T;
        if (n >= a.nk) continue;
        double t;
        int fl;
        float tau;
        if (stolt_point(a, q2, n, t, fl, tau)) {
            float2 x = rh[(size_t)rrow * a.nk + n];
            if (conj_in) x = cconj(x);
            V[n] = cmulc(x, modulation(a, Bl, n, t));
            G[n] = fl - kJ / 2;
            TAU[n] = tau;
            atomicMin(s_nev, n);
        } else {
            V[n] = c2(0.f, 0.f);
            G[n] = kGsentinel;
            TAU[n] = 0.f;
        }
    }
    __syncthreads();
    const int nev = *s_nev;
    float2 v[F::EPT];
    if (nev < a.nk) {
        const int base = G[nev] + 1;
        const int top = G[a.nk - 1] + kJ;
        // phase B: first contributing sample of every unwrapped cell in [base, top]
        for (int n = nev + threadIdx.x; n < a.nk; n += Cf::T) {
            const int from = n == nev ? base : G[n - 1] + kJ + 1;
            const int to = G[n] + kJ;
            for (int c = from; c <= to; ++c) LO[c - base] = (unsigned short)n;
        }
        __syncthreads();
        // phase C: gather into the cells this thread feeds to the FFT's first pass
#pragma unroll
        for (int i = 0; i < F::BPTO; ++i) {
            int cc, b;
            if (F::outer(i, cc, b)) {
#pragma unroll
                for (int j = 0; j < Cf::RO; ++j) {
                    const int g = b + j * Cf::SPAN;
                    float2 acc = c2(0.f, 0.f);
                    for (int cell = base + ((g - base) & (K - 1)); cell <= top; cell += K) {
                        for (int n = LO[cell - base]; n < a.nk && G[n] + 1 <= cell; ++n)
                            acc = cfmac(weight(wt, TAU[n], cell - G[n] - 1), V[n], acc);
                    }
                    v[i * Cf::RO + j] = acc;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < F::EPT; ++i) v[i] = c2(0.f, 0.f);
    }
    F::run(v, region, a.tw);        // opens with a barrier: phase C reads of the region are done
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int cc, b;
        if (F::outer(i, cc, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * Cf::SPAN;
                const int u = (x + a.mi + a.nk / 2) & (K - 1);
                if (u < a.nk) dst[u] = cscale(v[i * Cf::RO + j], a.sm[u]);
            }
        }
    }
    __syncthreads();
}

template <int K>
__global__ __launch_bounds__(NuCfg<K>::T) void k_nufft_adj(const float2* __restrict__ rh,
                                                           float2* __restrict__ ghat, NufftArgs a) {
    using Cf = NuCfg<K>;
    extern __shared__ float2 smem[];
    __shared__ int s_nev;
    float2* wt = smem;
    float2* region = smem + kWtabEntries;
    for (int i = threadIdx.x; i < kWtabEntries; i += Cf::T) wt[i] = a.wtab[i];
    const int b = blockIdx.x;
    if (b == 0) {
        adjoint_column<K>(a, rh, 0, false, 0, region, wt, ghat, &s_nev);
        if (a.nx >= 2) {
            const int ny = a.nx / 2;
            adjoint_column<K>(a, rh, ny, false, ny, region, wt, ghat + (size_t)ny * a.nk, &s_nev);
        }
    } else {
        adjoint_column<K>(a, rh, b, false, b, region, wt, ghat + (size_t)b * a.nk, &s_nev);
        adjoint_column<K>(a, rh, b, true, a.nx - b, region, wt, ghat + (size_t)(a.nx - b) * a.nk, &s_nev);
    }
}

template <typename Kern>
void set_lds(Kern kern, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int K>
hipError_t launch_fwd(const isam_plan_s* p, const float2* etahat, float2* zh, hipStream_t s) {
    using Cf = NuCfg<K>;
    set_lds(k_nufft_fwd<K>, Cf::LDS_FWD);
    hipLaunchKernelGGL(k_nufft_fwd<K>, dim3(std::max(1, p->nx / 2)), dim3(Cf::T), Cf::LDS_FWD, s, etahat, zh,
                       p->nufft_args());
    return hipGetLastError();
}

template <int K>
hipError_t launch_adj(const isam_plan_s* p, const float2* rh, float2* ghat, hipStream_t s) {
    using Cf = NuCfg<K>;
    set_lds(k_nufft_adj<K>, Cf::LDS_ADJ);
    hipLaunchKernelGGL(k_nufft_adj<K>, dim3(std::max(1, p->nx / 2)), dim3(Cf::T), Cf::LDS_ADJ, s, rh, ghat,
                       p->nufft_args());
    return hipGetLastError();
}

}  // namespace

#define ISAM_K_SWITCH(K_, CALL)                     \
    switch (K_) {                                   \
        case 32: { constexpr int K = 32; CALL; }    \
        case 64: { constexpr int K = 64; CALL; }    \
        case 128: { constexpr int K = 128; CALL; }  \
        case 256: { constexpr int K = 256; CALL; }  \
        case 512: { constexpr int K = 512; CALL; }  \
        case 1024: { constexpr int K = 1024; CALL; } \
        case 2048: { constexpr int K = 2048; CALL; } \
        case 4096: { constexpr int K = 4096; CALL; } \
        case 8192: { constexpr int K = 8192; CALL; } \
        default: return hipErrorInvalidValue;       \
    }

hipError_t nufft_fwd(const isam_plan_s* p, const float2* etahat, float2* zh, hipStream_t s) {
    ISAM_K_SWITCH(p->K, return launch_fwd<K>(p, etahat, zh, s));
}

hipError_t nufft_adj(const isam_plan_s* p, const float2* rh, float2* ghat, hipStream_t s) {
    ISAM_K_SWITCH(p->K, return launch_adj<K>(p, rh, ghat, s));
}

// Host replica of the Stolt span per column: the unwrapped cells [G_first + 1, G_last + J]
// must fit the LDS map of 2K entries (a margin of a few cells covers FP64 rounding
// differences between host and device at floor boundaries).
int nufft_span_ok(const isam_plan_s* p) {
    for (int i = 0; i < p->nx; ++i) {
        const int l = (i < (p->nx + 1) / 2) ? i : i - p->nx;
        const double q = 2.0 * 3.14159265358979323846 * l / (p->nx * p->g.dx);
        const double q2 = q * q;
        int first = -1;
        for (int n = 0; n < p->nk; ++n) {
            const double k = p->kc + (double)(n - p->nk / 2) * p->dk;
            if (4.0 * k * k - q2 > 0.0) {
                first = n;
                break;
            }
        }
        if (first < 0) continue;
        auto tpos = [&](int n) {
            const double k = p->kc + (double)(n - p->nk / 2) * p->dk;
            return std::floor(std::sqrt(4.0 * k * k - q2) * p->cT);
        };
        const double span = tpos(p->nk - 1) - tpos(first) + kJ;
        if (span + 4 > 2.0 * p->K) return 0;
        if (p->nk > 65535) return 0;
    }
    return 1;
}

}  // namespace isam
