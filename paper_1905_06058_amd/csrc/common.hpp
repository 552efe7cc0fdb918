// Shared device helpers for the ISAM kernels (complex float2 arithmetic, reductions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ISAM_DEV __device__ __forceinline__

ISAM_DEV float2 c2(float x, float y) { return make_float2(x, y); }
ISAM_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
ISAM_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Products are spelled out as one multiply and one fused multiply-add, so the rounding does
// not depend on which product the compiler would otherwise contract: every kernel that
// inlines these (a scan's own launch and a batch launch) rounds alike.
ISAM_DEV float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
ISAM_DEV float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
ISAM_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
ISAM_DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// acc += a * b
ISAM_DEV float2 cfma(float2 a, float2 b, float2 acc) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}
// acc += conj(a) * b
ISAM_DEV float2 cfmac(float2 a, float2 b, float2 acc) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(-a.y, b.x, acc.y);
    return acc;
}
ISAM_DEV float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }
// The FISTA gradient step eta - step * g (Alg. 1), one fused multiply-add per component:
// the adjoint's epilogue and the update pass form it alike.
ISAM_DEV float2 grad_step(float2 eta, float2 g, float step) {
    return make_float2(fmaf(-step, g.x, eta.x), fmaf(-step, g.y, eta.y));
}

// 64-wide wavefront sum by butterfly shuffles.
ISAM_DEV float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
ISAM_DEV float wave_max(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum of NV values per thread; threads 0..NV-1 write them to out[0..NV).
// `scratch` must hold NV * (T / 64) floats.  Ends with a barrier.
template <int T, int NV>
ISAM_DEV void block_sum_store(float (&v)[NV], float* scratch, float* out) {
    constexpr int NW = T / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        float s = wave_sum(v[i]);
        if (lane == 0) scratch[i * NW + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        float s = 0.f;
        for (int w = 0; w < NW; ++w) s += scratch[threadIdx.x * NW + w];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Internal arrays [rows][cols] exchanged between the lateral and the per-column passes use a
// column-blocked layout: blocks of 8 consecutive columns, each block stored row by row, so
// that a lateral tile of 8 columns is one contiguous run and a column is read in 64-byte
// (complex) segments.  Element (r, c) sits at blk(r, c, rows).
constexpr int kBlk = 8;
// 32-bit offsets: internal arrays hold fewer than 2^31 elements (nx * nk <= 2^23).
ISAM_DEV unsigned blk(int r, int c, int rows) { return ((unsigned)(c >> 3) * rows + r) * kBlk + (c & 7); }

// Maps launch order to tile order so that tiles sharing cache lines land on the
// same XCD: workgroups are dispatched round-robin over the 8 XCDs, so block b
// runs on XCD b % 8; consecutive tiles are given to blocks of one XCD.
ISAM_DEV int xcd_tile(int b, int nblocks) {
    constexpr int NXCD = 8;
    if (nblocks % NXCD) return b;
    const int per = nblocks / NXCD;
    return (b % NXCD) * per + b / NXCD;
}

// Tables of the direct image (Eq. 9) at index i < nk: D = e^{-j phi(k_i)} with
// phi = a2 d^2 + a3 d^3, d = (i - nk/2) dk (Eq. 7), and for row m = i - nk/2 the phase
// P = e^{-2 j kc dz m} (-1)^m / sqrt(nk) that turns an FFT over the sample index into the sum
// over e^{-2 j k_n z_m}.  FP64, arguments reduced mod 2 pi; no contraction, so every kernel
// that calls this stores the same bits.
ISAM_DEV void direct_table_entry(int i, int nk, double kc, double dk, double dz, double a2, double a3,
                                 float2& D, float2& P) {
#pragma clang fp contract(off)
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double d = (i - nk / 2) * dk;
    double phi = a2 * d * d + a3 * d * d * d;
    phi -= kTwoPi * rint(phi / kTwoPi);
    double sn, cs;
    sincos(-phi, &sn, &cs);
    D = make_float2((float)cs, (float)sn);
    const int m = i - nk / 2;
    double th = 2.0 * kc * dz * m;
    th -= kTwoPi * rint(th / kTwoPi);
    sincos(-th, &sn, &cs);
    const double norm = 1.0 / sqrt((double)nk);
    const double sg = (m & 1) ? -norm : norm;
    P = make_float2((float)(cs * sg), (float)(sn * sg));
}
