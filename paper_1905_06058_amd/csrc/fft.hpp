// LDS-resident Stockham FFT on CDNA4 wavefronts for lengths N = Q 2^P, Q in {1, 3, 5, 7}.
//
// A tile of C independent length-N sequences lives in LDS with element (x, c)
// at lds[lds_pad(x * LS + c)] (lds_size(N * LS) entries).  Passes use radices 2..16, plus
// one radix-Q pass (second in the sequence) when N has the odd factor Q; the first and the last pass
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
// Lengths N = Q 2^P (Q odd): the power-of-two schedule above with one radix-Q pass
// inserted after the first pass, so the first and last (outer) passes stay equal.
// fft_stride: product of the radices before a pass; fft_stage_off: offset of a pass
// (>= 1) in the staged twiddle table; fft_stage_len: the table's length.
constexpr int fft_odd(int n) { return (n & 1) || n == 0 ? n : fft_odd(n >> 1); }
constexpr int fft_p2(int n) { return ilog2(n / fft_odd(n)); }
constexpr int fft_np(int N, int L = 4) { return fft_npass(fft_p2(N), L) + (fft_odd(N) > 1 ? 1 : 0); }
constexpr int fft_radix(int N, int pass, int L = 4) {
    return fft_odd(N) == 1 ? 1 << fft_radix_log(fft_p2(N), pass, L)
           : pass == 0     ? 1 << fft_radix_log(fft_p2(N), 0, L)
           : pass == 1     ? fft_odd(N)
                           : 1 << fft_radix_log(fft_p2(N), pass - 1, L);
}
constexpr int fft_stride(int N, int pass, int L = 4) {
    return pass == 0 ? 1 : fft_stride(N, pass - 1, L) * fft_radix(N, pass - 1, L);
}
constexpr int fft_stage_off(int N, int pass, int L = 4) {
    return pass <= 1 ? 0 : fft_stage_off(N, pass - 1, L) + fft_radix(N, pass - 1, L) * fft_stride(N, pass - 1, L);
}
constexpr int fft_stage_len(int N, int L = 4) { return fft_np(N, L) <= 1 ? 1 : fft_stage_off(N, fft_np(N, L), L); }
// Lengths the schedule supports: Q in {1, 3, 5, 7}, and with Q > 1 at least two
// power-of-two passes (so that the outer passes exist).
constexpr bool fft_length_ok(int N, int L = 4) {
    return N >= 1 && (fft_odd(N) == 1 || ((fft_odd(N) == 3 || fft_odd(N) == 5 || fft_odd(N) == 7) &&
                                          fft_npass(fft_p2(N), L) >= 2));
}

// Entry e of the staged table of a length-N transform: (exponent, period) of the
// twiddle exp(-2 pi i exponent / period) it holds.
__host__ __device__ inline void fft_stage_entry(int N, int L, int e, int& expo, int& period) {
    const int np = fft_np(N, L);
    for (int p = 1; p < np; ++p) {
        const int R = fft_radix(N, p, L), NS = fft_stride(N, p, L);
        const int off = fft_stage_off(N, p, L);
        if (e >= off && e < off + R * NS) {
            expo = ((e - off) / NS) * ((e - off) % NS);
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
        return c2(fmaf(x.x, c, -(x.y * s)), fmaf(x.x, s, x.y * c));
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

// Odd radices R = 3, 5, 7: X_k = x_0 + sum_{n=1}^{H} (x_n + x_{R-n}) cos(2 pi n k / R)
// + i SIGN sum_{n=1}^{H} (x_n - x_{R-n}) sin(2 pi n k / R), H = (R - 1) / 2, and X_{R-k} the
// same with the sine part negated.  Tables hold cos / sin of 2 pi m / R, m < R.
__device__ constexpr float kCos3[3] = {1.0f, -0.5f, -0.5f};
__device__ constexpr float kSin3[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
__device__ constexpr float kCos5[5] = {1.0f, 0.30901699437494742f, -0.80901699437494742f, -0.80901699437494742f,
                                       0.30901699437494742f};
__device__ constexpr float kSin5[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f, -0.58778525229247313f,
                                       -0.95105651629515357f};
__device__ constexpr float kCos7[7] = {1.0f, 0.62348980185873353f, -0.22252093395631440f, -0.90096886790241913f,
                                       -0.90096886790241913f, -0.22252093395631440f, 0.62348980185873353f};
__device__ constexpr float kSin7[7] = {0.0f, 0.78183148246802981f, 0.97492791218182361f, 0.43388373911755812f,
                                       -0.43388373911755812f, -0.97492791218182361f, -0.78183148246802981f};
template <int R>
ISAM_DEV float odd_cos(int m) { return R == 3 ? kCos3[m] : R == 5 ? kCos5[m] : kCos7[m]; }
template <int R>
ISAM_DEV float odd_sin(int m) { return R == 3 ? kSin3[m] : R == 5 ? kSin5[m] : kSin7[m]; }

template <int R, int SIGN>
struct OddDft {
    ISAM_DEV static void run(float2* x) {
        constexpr int H = (R - 1) / 2;
        float2 a[H], d[H];
        float2 x0 = x[0], sum = x[0];
#pragma unroll
        for (int n = 1; n <= H; ++n) {
            a[n - 1] = cadd(x[n], x[R - n]);
            d[n - 1] = csub(x[n], x[R - n]);
            sum = cadd(sum, a[n - 1]);
        }
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            float2 re = x0, im = c2(0.f, 0.f);
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                const int m = (n * k) % R;
                re = c2(fmaf(a[n - 1].x, odd_cos<R>(m), re.x), fmaf(a[n - 1].y, odd_cos<R>(m), re.y));
                im = c2(fmaf(d[n - 1].x, odd_sin<R>(m), im.x), fmaf(d[n - 1].y, odd_sin<R>(m), im.y));
            }
            // i * SIGN * im
            const float2 t = SIGN > 0 ? c2(-im.y, im.x) : c2(im.y, -im.x);
            x[k] = cadd(re, t);
            x[R - k] = csub(re, t);
        }
        x[0] = sum;
    }
};
template <int SIGN>
struct Dft<3, SIGN> : OddDft<3, SIGN> {};
template <int SIGN>
struct Dft<5, SIGN> : OddDft<5, SIGN> {};
template <int SIGN>
struct Dft<7, SIGN> : OddDft<7, SIGN> {};

// Twiddle factor exp(SIGN * 2 pi i e / N) from the table of exp(-2 pi i e / N).
template <int SIGN>
ISAM_DEV float2 twiddle(const float2* tw, int e) {
    const float2 w = tw[e];
    return SIGN > 0 ? cconj(w) : w;
}

// PS: one LDS pad slot per 2^PS elements (lds_pad uses PS = 4).
template <int N, int C, int T, int SIGN, int LS = C, int L = 4, int PS = 4>
struct LdsFft {
    static_assert(fft_length_ok(N, L), "unsupported transform length");
    ISAM_DEV static constexpr int pad(int e) { return e + (e >> PS); }
    static constexpr int SIZE = N * LS + ((N * LS) >> PS) + 1;   // LDS entries used
    static constexpr int NP = fft_np(N, L);
    static constexpr int RO = fft_radix(N, 0, L);
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
            constexpr int R = fft_radix(N, PASS, L);
            constexpr int NS = fft_stride(N, PASS, L);
            constexpr int NB = N / R * C;
            constexpr int BPT = (NB + T - 1) / T;
            float2 x[BPT * R];
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int f = tid + i * T;
                if ((NB % T == 0) || f < NB) {
                    const int c = f % C, b = f / C;
#pragma unroll
                    for (int j = 0; j < R; ++j) x[i * R + j] = lds[pad((b + j * (N / R)) * LS + c)];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int f = tid + i * T;
                if ((NB % T == 0) || f < NB) {
                    const int c = f % C, b = f / C;
                    const int k = b % NS;
                    constexpr int OFF = fft_stage_off(N, PASS, L);
#pragma unroll
                    for (int j = 1; j < R; ++j)
                        x[i * R + j] = cmul(x[i * R + j], twiddle<SIGN>(tw, OFF + j * NS + k));
                    Dft<R, SIGN>::run(&x[i * R]);
                    const int base = (b - k) * R + k;
#pragma unroll
                    for (int j = 0; j < R; ++j) lds[pad((base + j * NS) * LS + c)] = x[i * R + j];
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
        run_head(v, lds, tw, tid);
        run_tail(v, lds, tw, tid);
    }

    // run() in two parts: every pass but the last (the data then sit in lds and v is free),
    // and the last pass (lds back to v), so that a caller can issue loads in between.
    ISAM_DEV static void run_head(float2 (&v)[EPT], float2* lds, const float2* tw, int tid) {
        if constexpr (NP == 1) {
#pragma unroll
            for (int i = 0; i < BPTO; ++i) Dft<RO, SIGN>::run(&v[i * RO]);
        } else if constexpr (NP > 1) {
            // first pass: no twiddles (stride 1), write Stockham order b*RO + j
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
                    Dft<RO, SIGN>::run(&v[i * RO]);
#pragma unroll
                    for (int j = 0; j < RO; ++j) lds[pad((b * RO + j) * LS + c)] = v[i * RO + j];
                }
            }
            __syncthreads();
            middle<1>(lds, tw, tid);
        }
    }

    ISAM_DEV static void run_tail(float2 (&v)[EPT], float2* lds, const float2* tw, int tid) {
        if constexpr (NP > 1) {
            // last pass: stride N/RO, twiddle exponent j*b, result stays in registers
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
#pragma unroll
                    for (int j = 0; j < RO; ++j) v[i * RO + j] = lds[pad((b + j * SPAN) * LS + c)];
                }
            }
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
                    constexpr int OFF = fft_stage_off(N, NP - 1, L);
#pragma unroll
                    for (int j = 1; j < RO; ++j) v[i * RO + j] = cmul(v[i * RO + j], twiddle<SIGN>(tw, OFF + j * SPAN + b));
                    Dft<RO, SIGN>::run(&v[i * RO]);
                }
            }
        }
    }
};

// Two-buffer form of LdsFft (same passes, same register layout, same twiddle table, LDS pad
// of one slot per 16 elements) for tiles whose LDS does not limit occupancy.  Pass p reads
// buffer (p - 1) & 1 and writes buffer p & 1, so each pass needs one barrier instead of two;
// the twiddles of every pass are fetched into registers once (Tw), so no table load waits
// behind a barrier, and a chained inverse and forward transform share one fetch (the inverse
// uses the conjugates).
template <int N, int C, int T, int L = 4>
struct LdsFft2 {
    using B = LdsFft<N, C, T, -1, C, L>;
    static constexpr int NP = B::NP, RO = B::RO, BPTO = B::BPTO, EPT = B::EPT, SPAN = B::SPAN;
    static constexpr int BUF = (B::SIZE + 1) & ~1;          // entries per buffer, 16-byte aligned
    static constexpr int SIZE = 2 * BUF;
    ISAM_DEV static constexpr int pad(int e) { return e + (e >> 4); }
    static constexpr int nb(int pass) { return N / fft_radix(N, pass, L) * C; }
    static constexpr int bpt(int pass) { return (nb(pass) + T - 1) / T; }
    // register offset of pass p's twiddles (middle passes 1..NP-2, then the last pass)
    static constexpr int tw_off(int pass) {
        return pass <= 1 ? 0 : tw_off(pass - 1) + bpt(pass - 1) * (fft_radix(N, pass - 1, L) - 1);
    }
    static constexpr int NTW = NP <= 1 ? 1 : tw_off(NP - 1) + BPTO * (RO - 1);
    struct Tw {
        float2 w[NTW];
    };

    ISAM_DEV static bool outer(int tid, int i, int& c, int& b) { return B::outer(tid, i, c, b); }

    template <int PASS>
    ISAM_DEV static void load_mid(const float2* __restrict__ tw, int tid, Tw& t) {
        if constexpr (PASS < NP - 1) {
            constexpr int R = fft_radix(N, PASS, L), NS = fft_stride(N, PASS, L);
            constexpr int OFF = fft_stage_off(N, PASS, L), TO = tw_off(PASS);
#pragma unroll
            for (int i = 0; i < bpt(PASS); ++i) {
                const int f = tid + i * T;
                const int k = (f / C) % NS;
#pragma unroll
                for (int j = 1; j < R; ++j)
                    t.w[TO + i * (R - 1) + j - 1] =
                        (nb(PASS) % T == 0 || f < nb(PASS)) ? tw[OFF + j * NS + k] : c2(0.f, 0.f);
            }
            load_mid<PASS + 1>(tw, tid, t);
        }
    }

    // The twiddles thread tid applies, for every pass (table of exp(-2 pi i e / period)).
    ISAM_DEV static void load(const float2* __restrict__ tw, int tid, Tw& t) {
        if constexpr (NP > 1) {
            load_mid<1>(tw, tid, t);
            constexpr int OFF = fft_stage_off(N, NP - 1, L), TO = tw_off(NP - 1);
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                const bool ok = outer(tid, i, c, b);
#pragma unroll
                for (int j = 1; j < RO; ++j)
                    t.w[TO + i * (RO - 1) + j - 1] = ok ? tw[OFF + j * SPAN + b] : c2(0.f, 0.f);
            }
        }
    }

    template <int SIGN>
    ISAM_DEV static float2 apply(float2 x, float2 w) {
        return cmul(x, SIGN > 0 ? cconj(w) : w);
    }

    template <int PASS, int SIGN>
    ISAM_DEV static void middle(float2* lds, const Tw& t, int tid) {
        if constexpr (PASS < NP - 1) {
            constexpr int R = fft_radix(N, PASS, L), NS = fft_stride(N, PASS, L), TO = tw_off(PASS);
            const float2* src = lds + ((PASS - 1) & 1) * BUF;
            float2* dst = lds + (PASS & 1) * BUF;
#pragma unroll
            for (int i = 0; i < bpt(PASS); ++i) {
                const int f = tid + i * T;
                if ((nb(PASS) % T == 0) || f < nb(PASS)) {
                    const int c = f % C, b = f / C;
                    const int k = b % NS;
                    float2 x[R];
#pragma unroll
                    for (int j = 0; j < R; ++j) x[j] = src[pad((b + j * (N / R)) * C + c)];
#pragma unroll
                    for (int j = 1; j < R; ++j) x[j] = apply<SIGN>(x[j], t.w[TO + i * (R - 1) + j - 1]);
                    Dft<R, SIGN>::run(x);
                    const int base = (b - k) * R + k;
#pragma unroll
                    for (int j = 0; j < R; ++j) dst[pad((base + j * NS) * C + c)] = x[j];
                }
            }
            __syncthreads();
            middle<PASS + 1, SIGN>(lds, t, tid);
        }
    }

    // As LdsFft::run, over lds[0, SIZE).  With open = false the opening barrier is left out:
    // the caller guarantees that no thread still reads buffer 0 (true after a transform of this
    // type when NP is odd, since its last pass reads buffer 1).  The caller places a barrier
    // before writing lds again afterwards.
    template <int SIGN>
    ISAM_DEV static void run(float2 (&v)[EPT], float2* lds, const Tw& t, int tid, bool open = true) {
        if constexpr (NP == 0) {
            return;
        } else if constexpr (NP == 1) {
#pragma unroll
            for (int i = 0; i < BPTO; ++i) Dft<RO, SIGN>::run(&v[i * RO]);
        } else {
            if (open) __syncthreads();
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
                    Dft<RO, SIGN>::run(&v[i * RO]);
#pragma unroll
                    for (int j = 0; j < RO; ++j) lds[pad((b * RO + j) * C + c)] = v[i * RO + j];
                }
            }
            __syncthreads();
            middle<1, SIGN>(lds, t, tid);
            const float2* src = lds + ((NP - 2) & 1) * BUF;
            constexpr int TO = tw_off(NP - 1);
#pragma unroll
            for (int i = 0; i < BPTO; ++i) {
                int c, b;
                if (outer(tid, i, c, b)) {
#pragma unroll
                    for (int j = 0; j < RO; ++j) v[i * RO + j] = src[pad((b + j * SPAN) * C + c)];
#pragma unroll
                    for (int j = 1; j < RO; ++j) v[i * RO + j] = apply<SIGN>(v[i * RO + j], t.w[TO + i * (RO - 1) + j - 1]);
                    Dft<RO, SIGN>::run(&v[i * RO]);
                }
            }
        }
    }
};

// LdsFft behind the interface of LdsFft2 (tiles too large for two buffers).
template <int N, int C, int T, int L = 4>
struct LdsFft1 {
    using B = LdsFft<N, C, T, -1, C, L>;
    static constexpr int NP = B::NP, RO = B::RO, BPTO = B::BPTO, EPT = B::EPT, SPAN = B::SPAN;
    static constexpr int SIZE = B::SIZE;
    struct Tw {
        const float2* p;
    };
    ISAM_DEV static bool outer(int tid, int i, int& c, int& b) { return B::outer(tid, i, c, b); }
    ISAM_DEV static void load(const float2* __restrict__ tw, int, Tw& t) { t.p = tw; }
    template <int SIGN>
    ISAM_DEV static void run(float2 (&v)[EPT], float2* lds, const Tw& t, int tid, bool /*open*/ = true) {
        LdsFft<N, C, T, SIGN, C, L>::run(v, lds, t.p, tid);
    }
};

}  // namespace isam
