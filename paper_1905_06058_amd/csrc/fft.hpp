// LDS-resident Stockham FFT for power-of-two lengths on CDNA4 wavefronts.
//
// A tile of C independent length-N sequences lives in LDS with element (x, c)
// at lds[lds_pad(x * LS + c)] (lds_size(N * LS) entries).  Passes use radices 2..16; the first and the last pass
// share one "outer" radix RO so that the register layout a thread holds after
// a transform (x = b + j N/RO for its butterflies b, j < RO) is exactly the
// layout the first pass of the next transform expects.  That lets kernels
// chain an inverse and a forward transform, or feed the first pass straight
// from global memory and consume the last pass straight to global memory,
// without an extra trip through LDS.
//
// DFT convention: X_k = sum_n x_n exp(SIGN * 2 pi i n k / N), unnormalised.
// Twiddles come from a staged table (fft_stage_table): for every pass p >= 1 with radix
// R and stride NS, the block [j][k] (j < R, k < NS) holds exp(-2 pi i j k / (NS R)), so
// the lanes of a wave (consecutive butterflies) read consecutive entries.
#pragma once
#include "common.hpp"

namespace isam {

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// LDS position of logical element L of a tile: one pad slot per 16 elements, so the
// power-of-two strides of the Stockham passes spread over all banks.
constexpr int lds_pad(int L) { return L + (L >> 4); }
constexpr int lds_size(int n) { return n + (n >> 4) + 1; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

// Pass structure of an N = 2^P transform with radices up to 2^L: outer radix 2^a at both
// ends, radix-2^L (and one smaller) passes in between.
constexpr int fft_npass(int P, int L = 4) {
    return P == 0 ? 0 : (P <= L ? 1 : 2 + (P - 2 * imin(L, P / 2) + L - 1) / L);
}
constexpr int fft_radix_log(int P, int pass, int L = 4) {
    if (P <= L) return P;
    const int a = imin(L, P / 2);
    const int np = fft_npass(P, L);
    if (pass == 0 || pass == np - 1) return a;
    const int rem = P - 2 * a - L * (pass - 1);
    return rem >= L ? L : rem;
}
constexpr int fft_stride_before(int P, int pass, int L = 4) {   // product of radices of passes < pass
    return pass == 0 ? 1 : fft_stride_before(P, pass - 1, L) * (1 << fft_radix_log(P, pass - 1, L));
}
// Offset of pass `pass` (>= 1) in the staged twiddle table, and the table's length.
constexpr int fft_stage_offset(int P, int pass, int L = 4) {
    return pass <= 1 ? 0
                     : fft_stage_offset(P, pass - 1, L) +
                           (1 << fft_radix_log(P, pass - 1, L)) * fft_stride_before(P, pass - 1, L);
}
constexpr int fft_stage_size(int P, int L = 4) {
    return fft_npass(P, L) <= 1 ? 1 : fft_stage_offset(P, fft_npass(P, L), L);
}

// Entry e of the staged table of a length-2^P transform: (exponent, period) of the
// twiddle exp(-2 pi i exponent / period) it holds.
inline void fft_stage_entry(int P, int L, int e, int& expo, int& period) {
    const int np = fft_npass(P, L);
    for (int p = 1; p < np; ++p) {
        const int R = 1 << fft_radix_log(P, p, L), NS = fft_stride_before(P, p, L);
        const int off = fft_stage_offset(P, p, L);
        if (e >= off && e < off + R * NS) {
            const int j = (e - off) / NS, k = (e - off) % NS;
            expo = j * k;
            period = NS * R;
            return;
        }
    }
    expo = 0;
    period = 1;
}

// cos / sin of 2 pi k / 16, k = 0..15
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// x * exp(SIGN * 2 pi i k / R), constant k and R <= 16
template <int R, int K, int SIGN>
ISAM_DEV float2 rot_const(float2 x) {
    constexpr int e = (K * (16 / R)) & 15;
    if constexpr (e == 0) return x;
    else if constexpr (e == 4) return SIGN > 0 ? c2(-x.y, x.x) : c2(x.y, -x.x);
    else if constexpr (e == 8) return c2(-x.x, -x.y);
    else if constexpr (e == 12) return SIGN > 0 ? c2(x.y, -x.x) : c2(-x.y, x.x);
    else {
        const float c = kCos16[e], s = SIGN * kSin16[e];
        return c2(x.x * c - x.y * s, x.x * s + x.y * c);
    }
}

// In-register DFT of R points (natural order in, natural order out).
template <int R, int SIGN>
struct Dft {
    template <int K>
    ISAM_DEV static void combine(float2* x, const float2* e, const float2* o) {
        if constexpr (K < R / 2) {
            const float2 t = rot_const<R, K, SIGN>(o[K]);
            x[K] = cadd(e[K], t);
            x[K + R / 2] = csub(e[K], t);
            combine<K + 1>(x, e, o);
        }
    }
    ISAM_DEV static void run(float2* x) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int n = 0; n < R / 2; ++n) {
            e[n] = x[2 * n];
            o[n] = x[2 * n + 1];
        }
        Dft<R / 2, SIGN>::run(e);
        Dft<R / 2, SIGN>::run(o);
        combine<0>(x, e, o);
    }
};
template <int SIGN>
struct Dft<1, SIGN> {
    ISAM_DEV static void run(float2*) {}
};
template <int SIGN>
struct Dft<2, SIGN> {
    ISAM_DEV static void run(float2* x) {
        const float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};
template <int SIGN>
struct Dft<4, SIGN> {
    ISAM_DEV static void run(float2* x) {
        const float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const float2 c = cadd(x[1], x[3]);
        const float2 d = rot_const<4, 1, SIGN>(csub(x[1], x[3]));
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};

// Twiddle factor exp(SIGN * 2 pi i e / N) from the table of exp(-2 pi i e / N).
template <int SIGN>
ISAM_DEV float2 twiddle(const float2* tw, int e) {
    const float2 w = tw[e];
    return SIGN > 0 ? cconj(w) : w;
}

template <int N, int C, int T, int SIGN, int LS = C, int L = 4>
struct LdsFft {
    static constexpr int P = ilog2(N);
    static constexpr int NP = fft_npass(P, L);
    static constexpr int RO = 1 << fft_radix_log(P, 0, L);
    static constexpr int NBO = N / RO * C;                  // butterflies in an outer pass
    static constexpr int BPTO = (NBO + T - 1) / T;          // per thread
    static constexpr int EPT = BPTO * RO;                   // register elements per thread
    static constexpr int SPAN = N / RO;                     // stride between taps of a butterfly

    // Butterfly f of an outer pass for thread tid: column and butterfly index.
    ISAM_DEV static bool outer(int tid, int i, int& c, int& b) {
        const int f = tid + i * T;
        c = f % C;
        b = f / C;
        return (NBO % T == 0) || f < NBO;
    }

    template <int PASS>
    ISAM_DEV static void middle(float2* lds, const float2* tw, int tid) {
        if constexpr (PASS < NP - 1) {
            constexpr int R = 1 << fft_radix_log(P, PASS, L);
            constexpr int NS = fft_stride_before(P, PASS, L);
            constexpr int NB = N / R * C;
            constexpr int BPT = (NB + T - 1) / T;
            float2 x[BPT * R];
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int f = tid + i * T;
                if ((NB % T == 0) || f < NB) {
                    const int c = f % C, b = f / C;
#pragma unroll
                    for (int j = 0; j < R; ++j) x[i * R + j] = lds[lds_pad((b + j * (N / R)) * LS + c)];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int f = tid + i * T;
                if ((NB % T == 0) || f < NB) {
                    const int c = f % C, b = f / C;
                    const int k = b % NS;
                    constexpr int OFF = fft_stage_offset(P, PASS, L);
#pragma unroll
                    for (int j = 1; j < R; ++j)
                        x[i * R + j] = cmul(x[i * R + j], twiddle<SIGN>(tw, OFF + j * NS + k));
                    Dft<R, SIGN>::run(&x[i * R]);
                    const int base = (b - k) * R + k;
#pragma unroll
                    for (int j = 0; j < R; ++j) lds[lds_pad((base + j * NS) * LS + c)] = x[i * R + j];
                }
            }
            __syncthreads();
            middle<PASS + 1>(lds, tw, tid);
        }
    }

    // Thread tid (0..T-1; threads of a larger block may run independent tiles with their
    // own lds) holds in v the inputs at x = b + j N/RO (butterfly i, tap j at v[i*RO + j]); on return it
    // holds the transform at the same positions.  Uses lds (N*LS entries) for N > 16: it
    // opens with a barrier (earlier readers of lds are done), and the caller must place a
    // barrier before writing lds again afterwards.
    ISAM_DEV static void run(float2 (&v)[EPT], float2* lds, const float2* tw, int tid) {
        if constexpr (NP == 0) {
            return;
        } else if constexpr (NP == 1) {
#pragma unroll
            for (int i = 0; i < BPTO; ++i) Dft<RO, SIGN>::run(&v[i * RO]);
        } else {
            // first pass: no twiddles (stride 1), write Stockham order b*RO + j
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
                    Dft<RO, SIGN>::run(&v[i * RO]);
#pragma unroll
                    for (int j = 0; j < RO; ++j) lds[lds_pad((b * RO + j) * LS + c)] = v[i * RO + j];
                }
            }
            __syncthreads();
            middle<1>(lds, tw, tid);
            // last pass: stride N/RO, twiddle exponent j*b, result stays in registers
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
#pragma unroll
                    for (int j = 0; j < RO; ++j) v[i * RO + j] = lds[lds_pad((b + j * SPAN) * LS + c)];
                }
            }
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
                    constexpr int OFF = fft_stage_offset(P, NP - 1, L);
#pragma unroll
                    for (int j = 1; j < RO; ++j) v[i * RO + j] = cmul(v[i * RO + j], twiddle<SIGN>(tw, OFF + j * SPAN + b));
                    Dft<RO, SIGN>::run(&v[i * RO]);
                }
            }
        }
    }
};

}  // namespace isam
