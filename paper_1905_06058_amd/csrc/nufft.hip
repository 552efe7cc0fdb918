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
// C2R lateral pass turns into Re(F^{-1} X) (Eq. 5), or, in the solver, the residual
// spectrum Z - F(y).
//
// Adjoint: the exact transpose, one lateral pair per workgroup (partners share their
// Stolt points and weights).  The transposed interpolation is formed without atomics (see
// nufft_adj_body): t_n increases by at least 2 per sample, so the contributions to a cell
// can be given fixed, single-writer slots.
#include <algorithm>

#include "common.hpp"
#include "fft.hpp"
#include "plan.hpp"

namespace isam {
namespace {

template <int K>
struct NuCfg {
    static constexpr int NK = K / 2;
    static constexpr int RO = fft_radix(K, 0);
    static constexpr int NB = K / RO;
    static constexpr int T = NB < 64 ? 64 : (NB > 256 ? 256 : NB);    // threads per column
    static constexpr int NPT = (NK + T - 1) / T;           // output samples per thread
    static constexpr int SPAN = K / RO;
    using Fwd = LdsFft<K, 1, T, +1>;
    // padded FFT buffer (float2), also holding Y with its J-entry wrap halo
    static constexpr int BUF = lds_size(K) > K + 8 ? lds_size(K) : K + 8;
    // forward: two columns in parallel (two halves of the block), shared weight table
    static constexpr size_t LDS_FWD = (size_t)(2 * BUF + kWtabEntries) * sizeof(float2);
    static_assert(LDS_FWD <= 160 * 1024, "forward tile exceeds the LDS of one CU");
};

// Adjoint: one lateral pair per block, T threads per column (radix-8 passes, so K/8 threads
// share a column).
// Samples are processed in chunks of CS; a chunk's cells fit SLOTC slots-triples.
template <int K>
struct NuAdjCfg {
    static constexpr int NK = K / 2;
    static constexpr int L = 3;
    static constexpr int RO = fft_radix(K, 0, L);
    static constexpr int NB = K / RO;
    static constexpr int T = NB < 64 ? 64 : (NB > 512 ? 512 : NB);
    static constexpr int SPAN = K / RO;
    static constexpr int CS = T < NK / 4 ? T : NK / 4;            // samples per chunk
    static constexpr int NCH = NK / CS;                             // chunks
    static constexpr int SLOTC = 2 * CS + CS / 8 + 16;             // cells of one chunk
    using Adj = LdsFft<K, 1, T, -1, 1, L, 6>;       // sparser padding: a smaller tile
    // per-half strides (float2) of the FFT tiles and of the slot arrays, 16-byte aligned
    static constexpr int TS = (Adj::SIZE + 1) & ~1;
    static constexpr int SLS = (3 * SLOTC + 1) & ~1;
    // Y' accumulates in registers (each thread owns the cells its FFT butterflies start from),
    // so the two halves' slot arrays and FFT tiles share one LDS region
    static constexpr size_t LDS =
        (size_t)(kWtabEntries + (2 * TS > 2 * SLS ? 2 * TS : 2 * SLS)) * sizeof(float2);
    static_assert(SLOTC < K, "a chunk's cells map to distinct oversampled cells");
    static_assert(LDS <= 160 * 1024, "adjoint tile exceeds the LDS of one CU");
    // waves per SIMD that the LDS admits (at most 8): the register budget asked of the compiler
    static constexpr int BPC = (int)((160 * 1024) / LDS);
    static constexpr int WPE_LDS = BPC * (2 * T / 64) / 4;
    static constexpr int WPE = WPE_LDS > 8 ? 8 : (WPE_LDS < 1 ? 1 : WPE_LDS);
    // operands fetched ahead of their use (the epilogue's before the last FFT pass, and in
    // the single-scan kernel the modulation factors at the start): measured at K = 4096,
    // whose register budget holds them; at other lengths, and for the modulation factors in
    // the batched kernel, they spill (K = 2048) or cost occupancy (K = 8192)
    static constexpr bool EPI_AHEAD = K == 4096;
};

// Stolt grid position of sample n of a column with q^2 = q2 (FP64).  Returns false on an
// evanescent sample (4 k^2 <= q^2).  t = kz dz K / (2 pi); fl = floor(t); tau = t - fl.
// At q = 0 the Stolt map is the identity (kz = 2k) and t advances by exactly osf = K / nk per
// sample: t = t0 + 2 (n - nk/2) with floor(t0) and t0 - floor(t0) decided once on the host, so
// consecutive samples sit exactly two cells apart whatever the rounding of t0.  Elsewhere
// kz is the FP64 square root below.  Every operation is spelled out (explicit fused
// multiply-adds, no contraction), so each kernel that inlines this, and the plan-time check of
// the adjoint's slot bounds (k_nufft_check), computes bit-identical positions.
ISAM_DEV bool stolt_point(const NufftArgs& a, double q2, int n, double& t, int& fl, float& tau) {
#pragma clang fp contract(off)
    if (q2 == 0.0) {
        fl = a.f0 + 2 * (n - a.nk / 2);
        tau = a.tau0;
        t = a.t0 + 2.0 * (n - a.nk / 2);
        return true;
    }
    const double k = fma((double)(n - a.nk / 2), a.dk, a.kc);
    const double tk = 2.0 * k;
    const double d = fma(tk, tk, -q2);
    if (!(d > 0.0)) return false;
    // sqrt(d): hardware reciprocal square root refined by one Newton step on the root
    // (relative error about the square of the estimate's)
    const double y = __builtin_amdgcn_rsq(d);
    const double s0 = d * y, h = 0.5 * y;
    t = fma(h, fma(-s0, s0, d), s0) * a.cT;
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
    const float4* row = reinterpret_cast<const float4*>(wt + p * kWtabPiece + jj * 4);
    const float4 a = row[0], b = row[1];     // (c0, c1), (c2, c3)
    float2 w;
    w.x = fmaf(fmaf(fmaf(b.z, x, b.x), x, a.z), x, a.x);
    w.y = fmaf(fmaf(fmaf(b.w, x, b.y), x, a.w), x, a.y);
    return w;
}

// The per-sample modulation B_l E_n f_n (f_n only with a fractional focal row).
ISAM_DEV float2 modulation(const NufftArgs& a, float2 En, float Bl, double t) {
    float2 e = cscale(En, Bl);
    if (a.has_frac) {
        double ph = a.mr_over_K * t;
        ph -= rint(ph);
        float s, c;
        sincospif(-2.0f * (float)ph, &s, &c);
        e = cmul(e, c2(c, s));
    }
    return e;
}

// Oversampled depth spectrum Y of column col into buf (natural order plus the J-entry wrap
// halo), by the K-point LDS FFT; ends with a barrier.
template <int K>
ISAM_DEV void fft_column(const NufftArgs& a, const float2* __restrict__ etahat, int col, float2* buf, int tid) {
    using Cf = NuCfg<K>;
    using F = typename Cf::Fwd;
    float2 v[F::EPT];
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(tid, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * Cf::SPAN;
                const int u = (x + a.mi + a.nk / 2) & (K - 1);      // depth index placed at x
                const int uc = u < a.nk ? u : 0;
                const float2 e = cscale(etahat[blk(col, uc, a.ncol)], a.sm[uc]);
                v[i * Cf::RO + j] = u < a.nk ? e : c2(0.f, 0.f);
            }
        }
    }
    F::run(v, buf, a.tw, tid);
    __syncthreads();
    // Y in natural order, plus a halo Y[K + i] = Y[i] so the J taps of a sample are contiguous
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int c, b;
        if (F::outer(tid, i, c, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * Cf::SPAN;
                buf[x] = v[i * Cf::RO + j];
                if (j == 0 && x < kJ) buf[K + x] = v[i * Cf::RO + j];
            }
        }
    }
    __syncthreads();
}

// The thread's samples n = tid + r T of column col: J-tap interpolation of Y (in buf) at the
// Stolt points, times the modulation.
template <int K>
ISAM_DEV void gather_column(const NufftArgs& a, int col, const float2* buf, const float2* wt,
                            float2 (&xt)[NuCfg<K>::NPT], int tid) {
    using Cf = NuCfg<K>;
    float2 en[Cf::NPT];                     // e^{i phi} e^{2 i k z_f} / sqrt(nz) of the thread's samples
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) en[r] = a.En[min(tid + r * Cf::T, a.nk - 1)];
    const double q2 = a.q2[col];
    const float Bl = a.Bl[col];
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = tid + r * Cf::T;
        float2 out = c2(0.f, 0.f);
        double t;
        int fl;
        float tau;
        if (n < a.nk && stolt_point(a, q2, n, t, fl, tau)) {
            const float2* y = buf + ((fl - kJ / 2 + 1) & (K - 1));   // tap j = 1 at g0 + 1
            float2 acc = c2(0.f, 0.f);
#pragma unroll
            for (int jj = 0; jj < kJ; ++jj) acc = cfma(weight(wt, tau, jj), y[jj], acc);
            out = cmul(acc, modulation(a, en[r], Bl, t));
        }
        xt[r] = out;
    }
}

// Block = two halves of T threads; half h transforms one column of the lateral pair
// (l, nx - l) (block 0: the self-paired l = 0 and l = nx/2), then half 0 writes the
// Hermitian combination.
// With yhat (the lateral spectrum of measured spectra, blocked half), the kernel writes the
// residual spectrum R = Z - yhat instead of Z: for a unitary lateral DFT F,
// F(Re F^{-1} X) is the Hermitian part Z of X, so the lateral transform of the residual
// Re(F^{-1} X) - y needs no transform at all.  Partials of ||r||^2 = sum_l w_l |R_l|^2
// (Parseval over the half spectrum, w = 1 at l = 0 and nx/2, else 2) go to partials.
// Body of workgroup bidx of nblk (one scan); the kernels below run it for a single scan or
// for the scans of a batch.
template <int K>
ISAM_DEV void nufft_fwd_body(const float2* __restrict__ etahat, const float2* __restrict__ yhat,
                             float2* __restrict__ zh, const NufftArgs& a, float* __restrict__ partials, int bidx,
                             int nblk) {
    using Cf = NuCfg<K>;
    if (a.stop && *a.stop) return;                     // solver already stopped (uniform)
    extern __shared__ float2 smem[];
    const int half = threadIdx.x / Cf::T, tid = threadIdx.x % Cf::T;
    float2* buf = smem + half * Cf::BUF;
    float2* wt = smem + 2 * Cf::BUF;
    for (int i = threadIdx.x; i < kWtabEntries; i += 2 * Cf::T) wt[i] = a.wtab[i];
    const int b = xcd_tile(bidx, nblk);                // neighbouring pairs on one XCD
    const FwdPair pr = a.pairs[b];
    const int col = half == 0 || pr.mode == 2 ? pr.a : pr.b;
    fft_column<K>(a, etahat, col, buf, tid);
    const int nh = a.nhalf;
    float acc[1] = {0.f};
    if (pr.mode == 0) {
        // Partners a, b = -a share q^2, hence the Stolt points, weights and modulation: each
        // of the 2T threads interpolates its samples of both columns with one set of weights
        // and forms the Hermitian combination at once.
        constexpr int T2 = 2 * Cf::T;
        constexpr int NP2 = (Cf::NK + T2 - 1) / T2;
        const int j = threadIdx.x;
        float2 en[NP2], ya[NP2], yb[NP2];
#pragma unroll
        for (int r = 0; r < NP2; ++r) {
            const int n = min(j + r * T2, a.nk - 1);
            en[r] = a.En[n];
            ya[r] = yhat ? yhat[blk(pr.ha, n, nh)] : c2(0.f, 0.f);
            yb[r] = yhat && pr.hb >= 0 ? yhat[blk(pr.hb, n, nh)] : c2(0.f, 0.f);
        }
        const double q2 = a.q2[pr.a];
        const float Bl = a.Bl[pr.a];
        const float2* bufA = smem;
        const float2* bufB = smem + Cf::BUF;
#pragma unroll
        for (int r = 0; r < NP2; ++r) {
            const int n = j + r * T2;
            if (n >= a.nk) continue;
            float2 xa = c2(0.f, 0.f), xb = c2(0.f, 0.f);
            double t;
            int fl;
            float tau;
            if (stolt_point(a, q2, n, t, fl, tau)) {
                const int g = (fl - kJ / 2 + 1) & (K - 1);               // tap j = 1 at g0 + 1
                float2 sa = c2(0.f, 0.f), sb = c2(0.f, 0.f);
#pragma unroll
                for (int jj = 0; jj < kJ; ++jj) {
                    const float2 w = weight(wt, tau, jj);
                    sa = cfma(w, bufA[g + jj], sa);
                    sb = cfma(w, bufB[g + jj], sb);
                }
                const float2 m = modulation(a, en[r], Bl, t);
                xa = cmul(sa, m);
                xb = cmul(sb, m);
            }
            const float2 zc = cscale(cadd(xa, cconj(xb)), 0.5f);
            const float2 z = csub(zc, ya[r]);
            zh[blk(pr.ha, n, nh)] = z;
            if (pr.hb >= 0) {                          // both stored: Z[b] = conj Z[a]
                const float2 z1 = csub(cconj(zc), yb[r]);
                zh[blk(pr.hb, n, nh)] = z1;
                acc[0] += cabs2(z) + cabs2(z1);
            } else {
                acc[0] += 2.f * cabs2(z);
            }
        }
    } else {
    float2 xt[Cf::NPT];
    gather_column<K>(a, col, buf, wt, xt, tid);
    float2 yh[Cf::NPT], yh1[Cf::NPT];
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = min(tid + r * Cf::T, a.nk - 1);
        yh[r] = yhat && half == 0 ? yhat[blk(pr.ha, n, nh)] : c2(0.f, 0.f);
        yh1[r] = yhat && half == 0 && pr.hb >= 0 ? yhat[blk(pr.hb, n, nh)] : c2(0.f, 0.f);
    }
    __syncthreads();
    if (half == 1) {
#pragma unroll
        for (int r = 0; r < Cf::NPT; ++r) {
            const int n = tid + r * Cf::T;
            if (n < a.nk) buf[n] = xt[r];
        }
    }
    __syncthreads();
    if (half == 0) {
        const float2* other = smem + Cf::BUF;
#pragma unroll
        for (int r = 0; r < Cf::NPT; ++r) {
            const int n = tid + r * Cf::T;
            if (n >= a.nk) continue;
            const float2 xb = other[n];
            if (pr.mode != 0) {                        // self-paired column(s): Z = Re X
                const float2 z0 = csub(c2(xt[r].x, 0.f), yh[r]);
                zh[blk(pr.ha, n, nh)] = z0;
                acc[0] += cabs2(z0);
                if (pr.mode == 1) {
                    const float2 z1 = csub(c2(xb.x, 0.f), yh1[r]);
                    zh[blk(pr.hb, n, nh)] = z1;
                    acc[0] += cabs2(z1);
                }
            } else {                                   // partners: Z[a] = (X[a] + conj X[b]) / 2
                const float2 zc = cscale(cadd(xt[r], cconj(xb)), 0.5f);
                const float2 z = csub(zc, yh[r]);
                zh[blk(pr.ha, n, nh)] = z;
                if (pr.hb >= 0) {                      // both stored: Z[b] = conj Z[a]
                    const float2 z1 = csub(cconj(zc), yh1[r]);
                    zh[blk(pr.hb, n, nh)] = z1;
                    acc[0] += cabs2(z) + cabs2(z1);
                } else {
                    acc[0] += 2.f * cabs2(z);
                }
            }
        }
    }
    }
    if (partials) {
        __syncthreads();
        block_sum_store<2 * Cf::T, 1>(acc, reinterpret_cast<float*>(smem), partials + b * kRedSlots);
    }
}

template <int K>
__global__ __launch_bounds__(2 * NuCfg<K>::T) void k_nufft_fwd(const float2* __restrict__ etahat,
                                                               const float2* __restrict__ yhat,
                                                               float2* __restrict__ zh, NufftArgs a,
                                                               float* __restrict__ partials) {
    nufft_fwd_body<K>(etahat, yhat, zh, a, partials, blockIdx.x, gridDim.x);
}

// Batched: workgroup b runs local workgroup map[b].y of scan map[b].x.
template <int K>
__global__ __launch_bounds__(2 * NuCfg<K>::T) void k_nufft_fwd_batch(const NuScan* __restrict__ scans,
                                                                     const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const NuScan& sc = scans[m.x];
    nufft_fwd_body<K>(sc.in, sc.in2, sc.out, sc.a, sc.partials, m.y, sc.nblk);
}

// Calibration gradient (Eq. 7, 13).  With theta = (a2, a3, z_f) the modulation obeys
// dc/dtheta = i D_theta c, D = ((k - k0)^2, (k - k0)^3, 2k - kz).  For real g and the unitary
// lateral DFT, <g, Re F^{-1}(c X)> = Re sum_{l,n} conj(G[l][n]) c X[l][n] with G = F g, so
//   d<g, A eta>/dtheta = -sum_{l,n} D_theta[l][n] Im(conj(G[l][n]) Xt[l][n]),   Xt = c X.
// Same column pairing as k_nufft_fwd; each half accumulates its own column (G[nx - l] =
// conj G[l] for real g) and the block writes three partial sums (slots 0..2).  ghalf is the
// blocked half spectrum of g (rows 0..nx/2).
template <int K>
__global__ __launch_bounds__(2 * NuCfg<K>::T) void k_nufft_calgrad(const float2* __restrict__ etahat,
                                                                   const float2* __restrict__ ghalf, NufftArgs a,
                                                                   float* __restrict__ partials) {
    using Cf = NuCfg<K>;
    extern __shared__ float2 smem[];
    const int half = threadIdx.x / Cf::T, tid = threadIdx.x % Cf::T;
    float2* buf = smem + half * Cf::BUF;
    float2* wt = smem + 2 * Cf::BUF;
    for (int i = threadIdx.x; i < kWtabEntries; i += 2 * Cf::T) wt[i] = a.wtab[i];
    const int b = blockIdx.x;
    const FwdPair pr = a.pairs[b];
    const bool active = half == 0 || pr.mode != 2;
    const int col = half == 0 || pr.mode == 2 ? pr.a : pr.b;
    float2 xt[Cf::NPT];
    fft_column<K>(a, etahat, col, buf, tid);
    gather_column<K>(a, col, buf, wt, xt, tid);
    const int nh = a.nhalf;
    // column b of a partner pair with no stored row has G[b] = conj G[a]
    const bool mirrored = half == 1 && pr.hb < 0;
    const int row = half == 0 || mirrored ? pr.ha : pr.hb;
    const double q2 = a.q2[col];
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < Cf::NPT; ++r) {
        const int n = tid + r * Cf::T;
        if (!active || n >= a.nk) continue;
        const double u = (double)(n - a.nk / 2) * a.dk;           // k - k0
        const double k2 = 2.0 * (a.kc + u);
        const double d = fma(k2, k2, -q2);
        if (!(d > 0.0)) continue;                                  // evanescent: c = 0
        float2 gl = ghalf[blk(row, n, nh)];
        if (mirrored) gl = cconj(gl);
        const float im = gl.x * xt[r].y - gl.y * xt[r].x;           // Im(conj(G) Xt)
        const double dz = q2 / (k2 + sqrt(d));                      // 2k - kz without cancellation
        acc[0] -= (float)(u * u) * im;
        acc[1] -= (float)(u * u * u) * im;
        acc[2] -= (float)dz * im;
    }
    __syncthreads();
    block_sum_store<2 * Cf::T, 3>(acc, reinterpret_cast<float*>(smem), partials + b * kRedSlots);
}

// Clears a half's slot arrays ([3][SLOTC] float2) with 16-byte stores (once, before the first
// chunk; afterwards each cell's reader clears its triple).
template <typename Cf>
ISAM_DEV void zero_slots(float2* SL, int tid) {
    constexpr int N2 = 3 * Cf::SLOTC, N4 = N2 / 2;
    float4* s4 = reinterpret_cast<float4*>(SL);
#pragma unroll
    for (int r = 0; r < (N4 + Cf::T - 1) / Cf::T; ++r) {
        const int i = tid + r * Cf::T;
        if (i < N4) s4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (N2 & 1) {
        if (tid == 0) SL[N2 - 1] = c2(0.f, 0.f);
    }
}

// Transposed NUFFT of the columns of one lateral pair per block (the pairs of the forward
// kernel: partners l and nx - l, or one or two self-paired columns).  A column reads its own
// half-spectrum row of the real residual's lateral transform, or, above nx/2, its partner's
// row conjugated.
//
// The transposed interpolation Y'[g] = sum over (n, j) with g0_n + j = g of
// conj(u_j(tau_n)) V_n is formed chunk by chunk without atomics: within a chunk every
// sample n writes its J products into a slot triple of its target cells, slot j / 2 of
// cell g0_n + 1 + j.  Two samples that reach one cell differ in g0 by at least 2, so they
// never share a slot: each slot has one writer.  Each cell then sums its three slots (in
// slot order) into Y'[cell mod K]; chunks follow one another, so every sum is formed in a
// fixed order and the result is bitwise repeatable.  A triple has one reader too (the
// thread that owns the cell), which clears it after reading: a chunk then needs two
// barriers (chunk base, scatter), since the next chunk's scatter comes after its first.
//
// Block = two halves of T threads; half h owns column h of the pair (its slots, its Y' in
// registers, its inverse FFT).  Partners share q^2, hence their Stolt points and weights:
// both halves take the same samples and half h evaluates taps 3h .. 3h + 2 for both
// columns.  Self-paired columns have their own q^2; each half then runs its own column
// with all J taps.
//
// In the FISTA loop (a.step_eta set) the output is the gradient step eta_hat - gstep g_hat
// of Alg. 1 rather than g_hat, so the update pass reads one array instead of two.
// EN_AHEAD: the modulation factors E_n of the thread's samples are fetched with its residual
// samples at the start, rather than in each chunk where the Stolt point is known.
template <int K, bool EN_AHEAD>
ISAM_DEV void nufft_adj_body(const float2* __restrict__ rh, float2* __restrict__ ghat, const NufftArgs& a,
                             int bidx, int nblk) {
    using Cf = NuAdjCfg<K>;
    using F = typename Cf::Adj;
    constexpr int T = Cf::T;
    static_assert(kJ == 6, "taps split 3 + 3 between the halves");
    if (a.stop && *a.stop) return;                     // solver already stopped (uniform)
    extern __shared__ float2 smem[];
    __shared__ int s_red[2][T / 64];
    const int half = threadIdx.x / T, tid = threadIdx.x % T;
    float2* wt = smem;
    float2* Y = smem + kWtabEntries + half * Cf::TS;                  // this half's FFT tile
    float2* SL0 = smem + kWtabEntries;                                // [2][SLS]: slots (same region)
    float2* SL = SL0 + half * Cf::SLS;
    // neighbouring pairs (which share cache lines of the blocked layout) on one XCD
    const FwdPair pr = a.pairs[xcd_tile(bidx, nblk)];
    const bool pair = pr.mode == 0;
    const bool live = half == 0 || pr.mode != 2;       // mode 2: a single self-paired column
    const int col = half == 0 ? pr.a : pr.b;
    for (int i = threadIdx.x; i < kWtabEntries; i += 2 * T) wt[i] = a.wtab[i];
    const int scol = pair ? pr.a : col;                // column whose Stolt points this half takes
    const double q2 = a.q2[scol];
    const float Bl = a.Bl[scol];
    // residual spectrum (of pr.a for a pair, else of the half's own column) of the thread's
    // samples, fetched up front.  The partner of a pair reads its own row
    // when it is stored (a volume's lx = 0 or nx/2 plane), else the conjugate of pr.a's.
    const int row0 = pair || !live || half == 0 ? pr.ha : pr.hb;
    float2 xr0[Cf::NCH], en0[EN_AHEAD ? Cf::NCH : 1];
#pragma unroll
    for (int ch = 0; ch < Cf::NCH; ++ch) {
        const int n = min(ch * Cf::CS + tid, a.nk - 1);
        xr0[ch] = live ? rh[blk(row0, n, a.nhalf)] : c2(0.f, 0.f);
        if constexpr (EN_AHEAD) en0[ch] = a.En[n];
    }
    // Y'[x] for the cells x = b + j K / RO this thread starts the inverse FFT from
    float2 v[F::EPT];
#pragma unroll
    for (int e = 0; e < F::EPT; ++e) v[e] = c2(0.f, 0.f);
    zero_slots<Cf>(SL, tid);
    for (int ch = 0; ch < Cf::NCH; ++ch) {
        const int n = ch * Cf::CS + tid;
        const bool mine = live && tid < Cf::CS;
        double t;
        int fl = 0;
        float tau = 0.f;
        const bool prop = mine && stolt_point(a, q2, n, t, fl, tau);
        float2 v0 = c2(0.f, 0.f), v1 = c2(0.f, 0.f);
        if (prop) {
            const float2 m = modulation(a, EN_AHEAD ? en0[EN_AHEAD ? ch : 0] : a.En[n], Bl, t);
            v0 = cmulc(xr0[ch], m);
            if (pair) v1 = cmulc(pr.hb >= 0 ? rh[blk(pr.hb, n, a.nhalf)] : cconj(xr0[ch]), m);
        }
        // chunk base: smallest g0 among the half's propagating samples.  t grows with n and
        // the evanescent samples come first, so within a wave it is the g0 of the first
        // propagating lane (read with every lane active, so that lane's value is current).
        const int g0v = fl - kJ / 2;
        const unsigned long long pm = __ballot(prop);
        const int g0w = pm ? __builtin_amdgcn_readlane(g0v, (int)__builtin_ctzll(pm)) : 0x7fffffff;
        if ((tid & 63) == 0) s_red[half][tid >> 6] = g0w;
        __syncthreads();
        int cbase = s_red[half][0];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) cbase = min(cbase, s_red[half][w]);
        const bool any = cbase != 0x7fffffff;
        if (prop) {
            // cell g0 + 1 + j (relative to cbase + 1), slot j / 2
            const int off = fl - kJ / 2 - cbase;
            const float tp = tau * kPieces;
            const int p = min((int)tp, kPieces - 1);
            const float xl = tp - (float)p;
            const float4* rowp = reinterpret_cast<const float4*>(wt + p * kWtabPiece);
            if (pair) {
                float2* d0 = SL0 + off;
                float2* d1 = SL0 + Cf::SLS + off;
#pragma unroll
                for (int k3 = 0; k3 < 3; ++k3) {
                    const int jj = 3 * half + k3;
                    const float4 ca = rowp[2 * jj], cb = rowp[2 * jj + 1];
                    float2 w;
                    w.x = fmaf(fmaf(fmaf(cb.z, xl, cb.x), xl, ca.z), xl, ca.x);
                    w.y = fmaf(fmaf(fmaf(cb.w, xl, cb.y), xl, ca.w), xl, ca.y);
                    d0[(jj >> 1) * Cf::SLOTC + jj] = cfmac(w, v0, c2(0.f, 0.f));
                    d1[(jj >> 1) * Cf::SLOTC + jj] = cfmac(w, v1, c2(0.f, 0.f));
                }
            } else {
                float2* d0 = SL + off;
#pragma unroll
                for (int jj = 0; jj < kJ; ++jj) {
                    const float4 ca = rowp[2 * jj], cb = rowp[2 * jj + 1];
                    float2 w;
                    w.x = fmaf(fmaf(fmaf(cb.z, xl, cb.x), xl, ca.z), xl, ca.x);
                    w.y = fmaf(fmaf(fmaf(cb.w, xl, cb.y), xl, ca.w), xl, ca.y);
                    d0[(jj >> 1) * Cf::SLOTC + jj] = cfmac(w, v0, c2(0.f, 0.f));
                }
            }
        }
        __syncthreads();
        if (any) {
            // cell x of this thread sits at c = x - (cbase + 1) (mod K) of the chunk's slots
#pragma unroll
            for (int i = 0; i < F::BPTO; ++i) {
                int cc, b;
                if (F::outer(tid, i, cc, b)) {
#pragma unroll
                    for (int j = 0; j < Cf::RO; ++j) {
                        const int c = (b + j * Cf::SPAN - cbase - 1) & (K - 1);
                        if (c < Cf::SLOTC) {
                            const float2 s0 = SL[c], s1 = SL[Cf::SLOTC + c], s2 = SL[2 * Cf::SLOTC + c];
                            v[i * Cf::RO + j] = cadd(v[i * Cf::RO + j], cadd(cadd(s0, s1), s2));
                            SL[c] = SL[Cf::SLOTC + c] = SL[2 * Cf::SLOTC + c] = c2(0.f, 0.f);
                        }
                    }
                }
            }
        }
    }
    F::run_head(v, Y, a.tw8, tid);    // opens with a barrier: the last reads of the slots are done
    // With EPI_AHEAD the epilogue's operands are fetched while the last pass runs (v is free
    // here: the data sit in LDS), so their latency hides behind the pass.
    static_assert(2 * Cf::NK == K, "the depth spectrum fills half of the oversampled grid");
    constexpr bool AH = Cf::EPI_AHEAD;
    // eta_hat of the gradient step
    float2 eh[AH ? F::EPT : 1];
    if (AH && a.step_eta && live) {
#pragma unroll
        for (int i = 0; i < F::BPTO; ++i) {
            int cc, b;
            if (F::outer(tid, i, cc, b)) {
#pragma unroll
                for (int j = 0; j < Cf::RO; ++j) {
                    const int u = (b + j * Cf::SPAN + a.mi + a.nk / 2) & (K - 1);
                    eh[AH ? i * Cf::RO + j : 0] = u < a.nk ? a.step_eta[blk(col, u, a.ncol)] : c2(0.f, 0.f);
                }
            }
        }
    }
    // the Kaiser-Bessel scales of the outputs kept: the depth indices u of a butterfly's RO
    // outputs share their residue mod K / RO, and (nk = K / 2) the RO / 2 of them below nk
    // are u = m K / RO + that residue, m < RO / 2.  Fetched at those indices, the loads issue
    // together rather than one per output branch.
    float smc[AH ? F::BPTO : 1][Cf::RO / 2];
    if constexpr (AH) {
#pragma unroll
        for (int i = 0; i < F::BPTO; ++i) {
            int cc, b;
            F::outer(tid, i, cc, b);
            const int r = (b + a.mi + a.nk / 2) & (Cf::SPAN - 1);
#pragma unroll
            for (int m = 0; m < Cf::RO / 2; ++m) smc[i][m] = a.sm[m * Cf::SPAN + r];
        }
    }
    F::run_tail(v, Y, a.tw8, tid);
    if (!live) return;
#pragma unroll
    for (int i = 0; i < F::BPTO; ++i) {
        int cc, b;
        if (F::outer(tid, i, cc, b)) {
#pragma unroll
            for (int j = 0; j < Cf::RO; ++j) {
                const int x = b + j * Cf::SPAN;
                const int u = (x + a.mi + a.nk / 2) & (K - 1);
                if (u < a.nk) {
                    const unsigned o = blk(col, u, a.ncol);
                    float sc;
                    if constexpr (AH) {
                        const int m = u / Cf::SPAN;
                        sc = smc[i][0];
#pragma unroll
                        for (int mm = 1; mm < Cf::RO / 2; ++mm) sc = m == mm ? smc[i][mm] : sc;
                    } else {
                        sc = a.sm[u];
                    }
                    const float2 g = cscale(v[i * Cf::RO + j], sc);
                    if (a.step_eta) ghat[o] = grad_step(AH ? eh[AH ? i * Cf::RO + j : 0] : a.step_eta[o], g, a.gstep);
                    else ghat[o] = g;
                }
            }
        }
    }
}

template <int K>
__global__ __launch_bounds__(2 * NuAdjCfg<K>::T, NuAdjCfg<K>::WPE) void k_nufft_adj(const float2* __restrict__ rh,
                                                              float2* __restrict__ ghat, NufftArgs a) {
    nufft_adj_body<K, NuAdjCfg<K>::EPI_AHEAD>(rh, ghat, a, blockIdx.x, gridDim.x);
}

template <int K>
__global__ __launch_bounds__(2 * NuAdjCfg<K>::T, NuAdjCfg<K>::WPE) void k_nufft_adj_batch(const NuScan* __restrict__ scans,
                                                                    const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    if (m.x < 0) return;                               // padding entry (uniform)
    const NuScan& sc = scans[m.x];
    nufft_adj_body<K, false>(sc.in, sc.out, sc.a, m.y, sc.nblk);      // registers: no room
}

template <typename Kern>
void set_lds(Kern kern, size_t bytes) {
    set_max_lds((const void*)kern, bytes);
}

template <int K>
hipError_t launch_fwd(const isam_plan_s* p, const float2* etahat, const float2* yhat, float2* zh, float* partials,
                      hipStream_t s, const int* stop) {
    using Cf = NuCfg<K>;
    set_lds(k_nufft_fwd<K>, Cf::LDS_FWD);
    NufftArgs a = p->nufft_args();
    a.stop = stop;
    ISAM_LAUNCH(k_nufft_fwd<K>, dim3(nufft_fwd_blocks(p)), dim3(2 * Cf::T), Cf::LDS_FWD, s, etahat,
                       yhat, zh, a, partials);
    return hipGetLastError();
}

template <int K>
hipError_t launch_calgrad(const isam_plan_s* p, const float2* etahat, const float2* ghalf, float* partials,
                          hipStream_t s) {
    using Cf = NuCfg<K>;
    set_lds(k_nufft_calgrad<K>, Cf::LDS_FWD);
    ISAM_LAUNCH(k_nufft_calgrad<K>, dim3(nufft_fwd_blocks(p)), dim3(2 * Cf::T), Cf::LDS_FWD, s, etahat, ghalf,
                p->nufft_args(), partials);
    return hipGetLastError();
}

template <int K>
hipError_t launch_adj(const isam_plan_s* p, const float2* rh, float2* ghat, hipStream_t s, const int* stop,
                      const float2* step_eta, float gstep) {
    using Cf = NuAdjCfg<K>;
    set_lds(k_nufft_adj<K>, Cf::LDS);
    NufftArgs a = p->nufft_args();
    a.stop = stop;
    a.step_eta = step_eta;
    a.gstep = gstep;
    ISAM_LAUNCH(k_nufft_adj<K>, dim3(nufft_adj_blocks(p)), dim3(2 * Cf::T), Cf::LDS, s, rh, ghat, a);
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

#define ISAM_K_SWITCH_INT(K_, CALL)                 \
    switch (K_) {                                   \
        case 32: { constexpr int K = 32; CALL; break; }    \
        case 64: { constexpr int K = 64; CALL; break; }    \
        case 128: { constexpr int K = 128; CALL; break; }  \
        case 256: { constexpr int K = 256; CALL; break; }  \
        case 512: { constexpr int K = 512; CALL; break; }  \
        case 1024: { constexpr int K = 1024; CALL; break; } \
        case 2048: { constexpr int K = 2048; CALL; break; } \
        case 4096: { constexpr int K = 4096; CALL; break; } \
        case 8192: { constexpr int K = 8192; CALL; break; } \
        default: return 0;                          \
    }

hipError_t nufft_fwd(const isam_plan_s* p, const float2* etahat, const float2* yhat, float2* zh, float* partials,
                     hipStream_t s, const int* stop) {
    ISAM_K_SWITCH(p->K, return launch_fwd<K>(p, etahat, yhat, zh, partials, s, stop));
}

hipError_t nufft_calgrad(const isam_plan_s* p, const float2* etahat, const float2* ghalf, float* partials,
                         hipStream_t s) {
    ISAM_K_SWITCH(p->K, return launch_calgrad<K>(p, etahat, ghalf, partials, s));
}

hipError_t nufft_adj(const isam_plan_s* p, const float2* rh, float2* ghat, hipStream_t s, const int* stop,
                     const float2* step_eta, float gstep) {
    ISAM_K_SWITCH(p->K, return launch_adj<K>(p, rh, ghat, s, stop, step_eta, gstep));
}

hipError_t nufft_fwd_batch(int K_, const NuScan* recs, const int2* map, int nblk, hipStream_t s) {
    ISAM_K_SWITCH(K_, {
        using Cf = NuCfg<K>;
        set_lds(k_nufft_fwd_batch<K>, Cf::LDS_FWD);
        hipLaunchKernelGGL(k_nufft_fwd_batch<K>, dim3(nblk), dim3(2 * Cf::T), Cf::LDS_FWD, s, recs, map);
        return hipGetLastError();
    });
}

hipError_t nufft_adj_batch(int K_, const NuScan* recs, const int2* map, int nblk, hipStream_t s) {
    ISAM_K_SWITCH(K_, {
        using Cf = NuAdjCfg<K>;
        set_lds(k_nufft_adj_batch<K>, Cf::LDS);
        hipLaunchKernelGGL(k_nufft_adj_batch<K>, dim3(nblk), dim3(2 * Cf::T), Cf::LDS, s, recs, map);
        return hipGetLastError();
    });
}

int nufft_fwd_blocks(const isam_plan_s* p) { return p->npairs; }
int nufft_adj_blocks(const isam_plan_s* p) { return p->npairs; }

namespace {

// The adjoint's transposed interpolation gives every (cell, slot) of a chunk one writer.  That
// holds if (1) consecutive propagating samples of a chunk have floor(t) at least 2 apart
// (dkz/dk >= 2 for any propagating component, exactly 2 at q = 0), and (2) the cells of a
// chunk, [g0_first + 1, g0_last + J], fit its slot array.  One thread per (column, chunk)
// walks the chunk's samples with stolt_point itself, so the check sees exactly the positions
// the kernels compute, and writes 1 into partials[col][chunk] if either bound fails, else 0.
template <int K>
__global__ __launch_bounds__(256) void k_nufft_check(NufftArgs a, float* __restrict__ partials) {
    using Cf = NuAdjCfg<K>;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.ncol * Cf::NCH) return;
    const int col = i / Cf::NCH, ch = i % Cf::NCH;
    const double q2 = a.q2[col];
    int first = 0, prev = 0;
    bool have = false, bad = false;
    for (int n = ch * Cf::CS; n < (ch + 1) * Cf::CS && n < a.nk; ++n) {
        double t;
        int fl;
        float tau;
        if (!stolt_point(a, q2, n, t, fl, tau)) continue;
        if (have && fl - prev < 2) bad = true;
        if (!have) first = fl;
        have = true;
        prev = fl;
    }
    if (have && prev - first + kJ > Cf::SLOTC) bad = true;
    partials[col * kRedSlots + ch] = bad ? 1.f : 0.f;
}

}  // namespace

namespace {

// Plan inspection: the Stolt points of one column exactly as the kernels compute them, and
// the weight table evaluated as the kernels evaluate it (testing and diagnostics).
__global__ void k_inspect_stolt(NufftArgs a, int col, int* __restrict__ fl_out, float* __restrict__ tau_out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.nk) return;
    double t;
    int fl = 0;
    float tau = 0.f;
    if (!stolt_point(a, a.q2[col], n, t, fl, tau)) {
        fl = -1;
        tau = -1.f;
    }
    fl_out[n] = fl;
    tau_out[n] = tau;
}

__global__ void k_inspect_weights(const float2* __restrict__ wtab, const float* __restrict__ tau, int n,
                                  float2* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float t = fminf(fmaxf(tau[i], 0.f), 0.99999994f);
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) out[i * kJ + jj] = weight(wtab, t, jj);
}

}  // namespace

hipError_t inspect_stolt(const isam_plan_s* p, int col, int* fl, float* tau, hipStream_t s) {
    hipLaunchKernelGGL(k_inspect_stolt, dim3((p->nk + 255) / 256), dim3(256), 0, s, p->nufft_args(), col, fl, tau);
    return hipGetLastError();
}

hipError_t inspect_weights(const isam_plan_s* p, const float* tau, int n, float2* out, hipStream_t s) {
    hipLaunchKernelGGL(k_inspect_weights, dim3((n + 255) / 256), dim3(256), 0, s, p->wtab, tau, n, out);
    return hipGetLastError();
}

hipError_t nufft_check(const isam_plan_s* p, float* partials, int* nslots, hipStream_t s) {
    ISAM_K_SWITCH(p->K, {
        const int n = p->ncol * NuAdjCfg<K>::NCH;
        *nslots = NuAdjCfg<K>::NCH;
        static_assert(NuAdjCfg<K>::NCH <= kRedSlots, "one flag per chunk in a partials row");
        hipLaunchKernelGGL(k_nufft_check<K>, dim3((n + 255) / 256), dim3(256), 0, s, p->nufft_args(), partials);
        return hipGetLastError();
    });
}

}  // namespace isam
