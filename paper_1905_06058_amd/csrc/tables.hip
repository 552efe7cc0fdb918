// Plan construction: validation, workspace, and the FP64 tables of the operator.
//
// Tables (all built on the device in FP64, stored in FP32 where the hot path reads them):
//   q_l^2, B(q_l)                       lateral frequencies and beam filter (Eq. 3, 16)
//   e^{i phi(k_n)} e^{2 i k_n z_f}      dispersion phase (Eq. 7, 13) and focal reference
//   s_m                                 Kaiser-Bessel scaling of the NUFFT
//   u_j(tau)                            min-max interpolation weights as a piecewise cubic in tau
//   twiddles                            staged per FFT pass for the depth and lateral FFTs
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "plan.hpp"

using namespace isam;

extern "C" const char* isam_strerror(int code) {
    switch (code) {
        case ISAM_OK: return "success";
        case ISAM_EINVAL: return "invalid argument";
        case ISAM_EALIAS: return "output aliases an input";
        case ISAM_EUNSUPPORTED: return "unsupported geometry or parameter";
        case ISAM_ENOMEM: return "device out of memory";
        case ISAM_ENODEV: return "no HIP device";
        case ISAM_EHIP: return "HIP runtime error";
        case ISAM_ENONFINITE: return "non-finite value in FISTA";
        default: return "unknown error";
    }
}

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

struct TableArgs {
    int nx, ny, nk, K;
    double dx, dy, waist, kc, dk, dz, a2, a3, zf, beta;
    double* q2;
    float* Bl;
    float2* En;
    float* sm;
    float2* Dn;
    float2* Pm;
};

// Kaiser-Bessel scaling s_m = Psi(0) / Psi(m / K), Psi(u) = sinh(a) / a, a = sqrt(beta^2 - (pi J u)^2).
__device__ double kb_scale(double m, int K, double beta) {
    const double u = m / K;
    const double a = sqrt(beta * beta - (kPi * kJ * u) * (kPi * kJ * u));
    return (sinh(beta) / beta) * (a / sinh(a));
}

__global__ void k_tables(TableArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.nx * a.ny) {
        // column i = lx * ny + ly; lateral frequencies in FFT order
        const int lx = i / a.ny, ly = i % a.ny;
        const int l = (lx < (a.nx + 1) / 2) ? lx : lx - a.nx;
        const int m = (ly < (a.ny + 1) / 2) ? ly : ly - a.ny;
        const double qx = 2.0 * kPi * l / (a.nx * a.dx);
        const double qy = a.ny > 1 ? 2.0 * kPi * m / (a.ny * a.dy) : 0.0;
        const double q2 = qx * qx + qy * qy;
        a.q2[i] = q2;
        a.Bl[i] = (float)exp(-q2 * a.waist * a.waist / 8.0);
    }
    if (i < a.nk) {
        const double d = (i - a.nk / 2) * a.dk;                   // k_n - k0
        const double k = a.kc + d;
        double psi = a.a2 * d * d + a.a3 * d * d * d + 2.0 * k * a.zf;   // Eq. 7 (a1 = 0) and focus
        psi -= 2.0 * kPi * rint(psi / (2.0 * kPi));
        double sn, cs;
        sincos(psi, &sn, &cs);
        const double norm = 1.0 / sqrt((double)a.nk);
        a.En[i] = make_float2((float)(cs * norm), (float)(sn * norm));
        a.sm[i] = (float)kb_scale(i - a.nk / 2, a.K, a.beta);
        direct_table_entry(i, a.nk, a.kc, a.dk, a.dz, a.a2, a.a3, a.Dn[i], a.Pm[i]);     // Eq. 9
    }
}

// Staged FFT twiddles (see fft.hpp) from a host-built (exponent, period) list, FP64.
__global__ void k_twiddles(const int2* __restrict__ ep, int n, float2* __restrict__ tw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double sn, cs;
        sincospi(-2.0 * ep[i].x / ep[i].y, &sn, &cs);
        tw[i] = make_float2((float)cs, (float)sn);
    }
}

// Sums over the object rows m in [-nz/2, nz/2) needed by the least-squares system
// of the min-max interpolator:
//   rho(x)  = sum_m s_m exp(2 pi i x m / K)       at x = tau + J/2 - j  (C^H b)
//   gram(d) = sum_m s_m^2 exp(2 pi i d m / K)     for d in (-J, J)      (C^H C)
// One block per value, FP64 tree reduction.
struct SumArgs {
    int nk, K;
    double beta;
    double nodes[4];        // cubic fit nodes in a piece, local coordinate in [0, 1]
    double* out;            // [(nrho + ngram) * 2]
};

__global__ void k_minmax_sums(SumArgs a) {
    constexpr int nrho = kPieces * 4 * kJ;
    const int b = blockIdx.x;
    double x;
    int power;
    if (b < nrho) {
        const int nd = b / kJ, j = b % kJ + 1;
        const int p = nd / 4, node = nd % 4;
        const double tau = (p + a.nodes[node]) / kPieces;
        x = tau + kJ / 2 - j;
        power = 1;
    } else {
        x = (b - nrho) - (kJ - 1);
        power = 2;
    }
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < a.nk; i += blockDim.x) {
        const double m = i - a.nk / 2;
        double s = kb_scale(m, a.K, a.beta);
        if (power == 2) s *= s;
        double sn, cs;
        sincospi(2.0 * x * m / a.K, &sn, &cs);
        re += s * cs;
        im += s * sn;
    }
    __shared__ double sre[256], sim[256];
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sre[threadIdx.x] += sre[threadIdx.x + w];
            sim[threadIdx.x] += sim[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.out[2 * b] = sre[0];
        a.out[2 * b + 1] = sim[0];
    }
}

struct FitArgs {
    int K, mi;
    double nodes[4];
    double vinv[16];        // inverse Vandermonde of the nodes: coef[q] = sum_i vinv[q*4+i] f(node_i)
    const double* sums;
    float2* wtab;
};

// Per piece: solve (C^H C) u = C^H b(tau) at the four nodes by complex Cholesky,
// apply the focal phase exp(-2 pi i mi (tau + J/2 - j) / K), fit a cubic per tap.
__global__ void k_minmax_fit(FitArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kPieces) return;
    constexpr int nrho = kPieces * 4 * kJ;
    double Lr[kJ][kJ], Li[kJ][kJ];
    // G[r][c] = gram(c - r); Cholesky G = L L^H (lower L, real positive diagonal)
    for (int r = 0; r < kJ; ++r) {
        for (int c = 0; c <= r; ++c) {
            const int d = c - r + (kJ - 1);
            double gr = a.sums[2 * (nrho + d)], gi = a.sums[2 * (nrho + d) + 1];
            // subtract sum_k L[r][k] conj(L[c][k])
            for (int k = 0; k < c; ++k) {
                gr -= Lr[r][k] * Lr[c][k] + Li[r][k] * Li[c][k];
                gi -= Li[r][k] * Lr[c][k] - Lr[r][k] * Li[c][k];
            }
            if (r == c) {
                Lr[r][r] = sqrt(gr);
                Li[r][r] = 0.0;
            } else {
                Lr[r][c] = gr / Lr[c][c];
                Li[r][c] = gi / Lr[c][c];
            }
        }
    }
    double ur[4][kJ], ui[4][kJ];
    for (int node = 0; node < 4; ++node) {
        const int nd = p * 4 + node;
        double yr[kJ], yi[kJ];
        for (int r = 0; r < kJ; ++r) {            // forward substitution L y = rho
            double sr = a.sums[2 * (nd * kJ + r)], si = a.sums[2 * (nd * kJ + r) + 1];
            for (int k = 0; k < r; ++k) {
                sr -= Lr[r][k] * yr[k] - Li[r][k] * yi[k];
                si -= Lr[r][k] * yi[k] + Li[r][k] * yr[k];
            }
            yr[r] = sr / Lr[r][r];
            yi[r] = si / Lr[r][r];
        }
        for (int r = kJ - 1; r >= 0; --r) {       // back substitution L^H u = y
            double sr = yr[r], si = yi[r];
            for (int k = r + 1; k < kJ; ++k) {     // (L^H)[r][k] = conj(L[k][r])
                sr -= Lr[k][r] * ur[node][k] + Li[k][r] * ui[node][k];
                si -= Lr[k][r] * ui[node][k] - Li[k][r] * ur[node][k];
            }
            ur[node][r] = sr / Lr[r][r];
            ui[node][r] = si / Lr[r][r];
        }
        const double tau = (p + a.nodes[node]) / kPieces;
        for (int r = 0; r < kJ; ++r) {
            const int j = r + 1;
            // phase exp(-2 pi i mi (tau + J/2 - j) / K), argument reduced exactly in the integer part
            const long long ip = ((long long)a.mi * (kJ / 2 - j)) % a.K;
            const double ang = -2.0 * ((double)ip + a.mi * tau) / a.K;
            double sn, cs;
            sincospi(ang, &sn, &cs);
            const double xr = ur[node][r] * cs - ui[node][r] * sn;
            const double xi = ur[node][r] * sn + ui[node][r] * cs;
            ur[node][r] = xr;
            ui[node][r] = xi;
        }
    }
    for (int r = 0; r < kJ; ++r) {
        for (int q = 0; q < 4; ++q) {
            double cr = 0.0, ci = 0.0;
            for (int node = 0; node < 4; ++node) {
                cr += a.vinv[q * 4 + node] * ur[node][r];
                ci += a.vinv[q * 4 + node] * ui[node][r];
            }
            a.wtab[p * kWtabPiece + r * 4 + q] = make_float2((float)cr, (float)ci);
        }
    }
    for (int e = kJ * 4; e < kWtabPiece; ++e) a.wtab[p * kWtabPiece + e] = make_float2(0.f, 0.f);
}

// Chebyshev nodes of [0, 1] and the inverse of their Vandermonde matrix (Gauss-Jordan, FP64).
void cubic_nodes(double nodes[4], double vinv[16]) {
    double V[4][8];
    for (int i = 0; i < 4; ++i) {
        nodes[i] = 0.5 * (1.0 - cos((2 * i + 1) * kPi / 8.0));
        double x = 1.0;
        for (int k = 0; k < 4; ++k) {
            V[i][k] = x;
            x *= nodes[i];
            V[i][4 + k] = (i == k) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(V[r][c]) > fabs(V[piv][c])) piv = r;
        for (int k = 0; k < 8; ++k) std::swap(V[c][k], V[piv][k]);
        const double d = V[c][c];
        for (int k = 0; k < 8; ++k) V[c][k] /= d;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            const double f = V[r][c];
            for (int k = 0; k < 8; ++k) V[r][k] -= f * V[c][k];
        }
    }
    // V^{-1}[q][i] maps values at nodes to monomial coefficient q
    for (int q = 0; q < 4; ++q)
        for (int i = 0; i < 4; ++i) vinv[q * 4 + i] = V[q][4 + i];
}

// Lateral-frequency columns (Eq. 2 over one or two lateral axes): column col = lx * ny + ly;
// the Hermitian half keeps lx <= nx/2 at the same index.  The partner of (lx, ly) is
// (-lx mod nx, -ly mod ny).  NUFFT workgroups (forward and adjoint): first the self-paired
// columns, two per workgroup, then one partner pair per workgroup.
void build_columns(const isam_plan_s* p, std::vector<isam::FwdPair>& pairs) {
    const int nx = p->nx, ny = p->ny, nh = p->nhalf;
    auto partner = [&](int c) { return ((nx - c / ny) % nx) * ny + (ny - c % ny) % ny; };
    std::vector<int> self;
    for (int c = 0; c < nh; ++c)
        if (partner(c) == c) self.push_back(c);
    for (size_t i = 0; i < self.size(); i += 2) {
        if (i + 1 < self.size())
            pairs.push_back({self[i], self[i + 1], self[i], self[i + 1], 1});
        else
            pairs.push_back({self[i], self[i], self[i], -1, 2});
    }
    for (int c = 0; c < nh; ++c) {
        const int q = partner(c);
        if (q == c) continue;
        if (q < nh) {
            if (c < q) pairs.push_back({c, q, c, q, 0});
        } else {
            pairs.push_back({c, q, c, -1, 0});
        }
    }
}

int validate(const isam_geometry* g) {
    if (!g) return ISAM_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->nk < 2) return ISAM_EINVAL;
    if (g->J < 2 || g->J > 16 || (g->J & 1)) return ISAM_EINVAL;
    if (g->osf < 1) return ISAM_EINVAL;
    if ((g->nk & 1) || g->nk < 2 * g->J) return ISAM_EINVAL;
    const double vals[] = {g->dx, g->lambda_c, g->dlambda, g->waist, g->z_focus, g->a2, g->a3,
                           g->kb_beta};
    for (double v : vals)
        if (!std::isfinite(v)) return ISAM_EINVAL;
    if (!(g->dx > 0) || !(g->lambda_c > 0) || !(g->dlambda > 0) || g->waist < 0) return ISAM_EINVAL;
    if (!(g->dlambda < g->lambda_c)) return ISAM_EINVAL;
    if (g->ny > 1 && (!std::isfinite(g->dy) || !(g->dy > 0))) return ISAM_EINVAL;
    if (g->ny > 1 && !lat_supported(g->ny)) return ISAM_EUNSUPPORTED;
    if ((int64_t)g->nx * g->ny * g->nk > ((int64_t)1 << 30)) return ISAM_EUNSUPPORTED;   // 32-bit offsets
    if (g->J != kJ || g->osf != 2) return ISAM_EUNSUPPORTED;
    if (!lat_supported(g->nx)) return ISAM_EUNSUPPORTED;
    if (!is_pow2(g->nk) || g->nk > 4096) return ISAM_EUNSUPPORTED;
    const double beta = g->kb_beta > 0 ? g->kb_beta : 2.34 * g->J;
    if (!(beta > kPi * g->J / (2.0 * g->osf))) return ISAM_EINVAL;   // scaling defined on all rows
    return ISAM_OK;
}

void derive(isam_plan_s* p, const isam_geometry* g) {
    p->g = *g;
    p->nx = g->nx;
    p->nk = g->nk;
    p->K = g->osf * g->nk;
    p->nh = g->nx / 2 + 1;
    p->ny = g->ny;
    p->ncol = g->nx * g->ny;
    p->nhalf = p->nh * g->ny;
    p->kc = 2.0 * kPi / g->lambda_c;
    p->band = 2.0 * kPi * g->dlambda / (g->lambda_c * g->lambda_c);
    p->dk = p->band / g->nk;
    p->dz = kPi / p->band;
    p->cT = p->dz * p->K / (2.0 * kPi);
    p->beta = g->kb_beta > 0 ? g->kb_beta : 2.34 * g->J;
    p->mf = g->z_focus / p->dz;
    p->mi = (int)std::lrint(p->mf);
    p->mr = p->mf - p->mi;
    if (std::fabs(p->mr) < 1e-9) p->mr = 0.0;
    // Stolt position of the centre sample at q = 0 (kz = 2 kc); the q = 0 column advances by
    // exactly osf cells per sample from it.  A position within 1e-9 of a grid point is put on
    // it (an integer lambda_c / dlambda puts every q = 0 sample on the grid).
    p->t0 = 2.0 * p->kc * p->cT;
    if (std::fabs(p->t0 - std::rint(p->t0)) < 1e-9) p->t0 = std::rint(p->t0);
    p->f0 = (int)std::floor(p->t0);
}

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return ISAM_EHIP;    \
    } while (0)

int build_twiddles(isam_plan_s* p, hipStream_t s) {
    // staged tables: depth FFT (radix caps 16 and 8), lateral FFT (caps 4, 8, 16), and for a
    // volume the y transform
    struct Item { int N, L; float2* dst; };
    std::vector<Item> items = {{p->K, 4, p->twK}, {p->K, 3, p->twK8}, {p->nx, 2, p->twX[2]}, {p->nx, 3, p->twX[3]},
                               {p->nx, 4, p->twX[4]}, {p->nk, 4, p->twN}};
    if (p->ny > 1)       // the y transform of a volume
        for (int L = 2; L <= 4; ++L) items.push_back({p->ny, L, p->twY[L]});
    int ntot = 0;
    for (const Item& it : items) ntot += fft_stage_len(it.N, it.L);
    int2* h = nullptr;
    if (hipHostMalloc((void**)&h, (size_t)ntot * sizeof(int2)) != hipSuccess) return ISAM_ENOMEM;
    int off = 0;
    for (const Item& it : items) {
        const int n = fft_stage_len(it.N, it.L);
        for (int e = 0; e < n; ++e) fft_stage_entry(it.N, it.L, e, h[off + e].x, h[off + e].y);
        off += n;
    }
    int2* d = nullptr;
    int rc = ISAM_OK;
    if (hipMalloc((void**)&d, (size_t)ntot * sizeof(int2)) != hipSuccess) rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipMemcpyAsync(d, h, (size_t)ntot * sizeof(int2), hipMemcpyHostToDevice, s) != hipSuccess)
        rc = ISAM_EHIP;
    off = 0;
    for (const Item& it : items) {
        const int n = fft_stage_len(it.N, it.L);
        if (rc == ISAM_OK) {
            hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, d + off, n, it.dst);
            if (hipGetLastError() != hipSuccess) rc = ISAM_EHIP;
        }
        off += n;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == ISAM_OK) rc = ISAM_EHIP;
    if (d) (void)hipFree(d);
    (void)hipHostFree(h);
    return rc;
}

int build_calibrated_tables(isam_plan_s* p, hipStream_t s) {
    TableArgs a;
    a.nx = p->nx;
    a.ny = p->ny;
    a.nk = p->nk;
    a.K = p->K;
    a.dx = p->g.dx;
    a.dy = p->g.dy;
    a.waist = p->g.waist;
    a.kc = p->kc;
    a.dk = p->dk;
    a.dz = p->dz;
    a.a2 = p->g.a2;
    a.a3 = p->g.a3;
    a.zf = p->g.z_focus;
    a.beta = p->beta;
    a.q2 = p->q2;
    a.Bl = p->Bl;
    a.En = p->En;
    a.sm = p->sm;
    a.Dn = p->Dn;
    a.Pm = p->Pm;
    const int n = std::max(p->ncol, p->nk);
    hipLaunchKernelGGL(k_tables, dim3((n + 255) / 256), dim3(256), 0, s, a);
    HIP_TRY(hipGetLastError());

    SumArgs sa;
    sa.nk = p->nk;
    sa.K = p->K;
    sa.beta = p->beta;
    FitArgs fa;
    cubic_nodes(fa.nodes, fa.vinv);
    std::memcpy(sa.nodes, fa.nodes, sizeof(sa.nodes));
    sa.out = p->wscratch;
    const int nsums = kPieces * 4 * kJ + (2 * kJ - 1);
    hipLaunchKernelGGL(k_minmax_sums, dim3(nsums), dim3(256), 0, s, sa);
    HIP_TRY(hipGetLastError());
    fa.K = p->K;
    fa.mi = p->mi;
    fa.sums = p->wscratch;
    fa.wtab = p->wtab;
    hipLaunchKernelGGL(k_minmax_fit, dim3(1), dim3(64), 0, s, fa);
    HIP_TRY(hipGetLastError());
    return ISAM_OK;
}

// Failure injection for tests of the clean-up path: with the environment variable
// ISAM_FAIL_ALLOC=n (n >= 1) set when isam_plan starts, that call's n-th table or workspace
// allocation fails as if the device were out of memory.  Read once per isam_plan call.
thread_local int g_fail_alloc = 0;

template <typename T>
int dalloc(T** ptr, size_t n) {
    if (g_fail_alloc > 0 && --g_fail_alloc == 0) {
        *ptr = nullptr;
        return ISAM_ENOMEM;
    }
    if (hipMalloc((void**)ptr, n * sizeof(T)) != hipSuccess) {
        *ptr = nullptr;
        return ISAM_ENOMEM;
    }
    return ISAM_OK;
}

}  // namespace

namespace isam {

void set_max_lds(const void* kern, size_t bytes) {
    if (bytes <= 65536) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    // kernels (and devices) whose limit is already raised: the attribute call then costs
    // nothing on the launch path
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> done;
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& d : done)
        if (d.first == kern && d.second == dev) return;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        done.emplace_back(kern, dev);
}

}  // namespace isam

namespace {

void release(isam_plan_s* p) {
    void* ptrs[] = {p->q2, p->Bl, p->En, p->sm, p->wtab, p->twK, p->twK8, p->twX[2], p->twX[3], p->twX[4],
                    p->twY[2], p->twY[3], p->twY[4], p->pairs, p->wscratch, p->twN, p->Dn, p->Pm, p->hist,
                    p->etahat, p->zh, p->rh, p->ghat, p->fista_hat, p->yhat, p->vec, p->sbuf, p->wbuf, p->zblk,
                    p->xs, p->xsh, p->red.partials, p->red.sums};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p->host_sums) (void)hipHostFree(p->host_sums);
    if (p->stop) (void)hipFree(p->stop);
    if (p->host_stop) (void)hipHostFree(p->host_stop);
    for (int i = 0; i < 2 * p->tev_cap; ++i)
        if (p->tev[i]) (void)hipEventDestroy(p->tev[i]);
    delete[] p->tev;
    delete[] p->ttag;
    delete p;
}

// The adjoint's single-writer slot bounds, checked on the device with the kernels' own Stolt
// arithmetic (nufft_check): EUNSUPPORTED if any (column, chunk) breaks them.  Synchronises.
int check_stolt(isam_plan_s* p, hipStream_t s) {
    int nslots = 0;
    HIP_TRY(isam::nufft_check(p, p->red.partials, &nslots, s));
    std::vector<float> flags((size_t)p->ncol * kRedSlots);
    HIP_TRY(hipMemcpyAsync(flags.data(), p->red.partials, flags.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < p->ncol; ++c)
        for (int ch = 0; ch < nslots; ++ch)
            if (flags[(size_t)c * kRedSlots + ch] != 0.f) return ISAM_EUNSUPPORTED;
    return ISAM_OK;
}

}  // namespace

isam::NufftArgs isam_plan_s::nufft_args() const {
    isam::NufftArgs a;
    a.nx = nx;
    a.nk = nk;
    a.K = K;
    a.mi = mi;
    a.has_frac = mr != 0.0;
    a.mr_over_K = mr / K;
    a.kc = kc;
    a.dk = dk;
    a.cT = cT;
    a.f0 = f0;
    a.tau0 = (float)(t0 - f0);
    a.t0 = t0;
    a.q2 = q2;
    a.Bl = Bl;
    a.En = En;
    a.sm = sm;
    a.wtab = wtab;
    a.tw = twK;
    a.tw8 = twK8;
    a.stop = nullptr;
    a.ncol = ncol;
    a.nhalf = nhalf;
    a.pairs = pairs;
    return a;
}

extern "C" int isam_plan(const isam_geometry* g, void* stream, isam_plan_t* out) {
    if (!out) return ISAM_EINVAL;
    *out = nullptr;
    int rc = validate(g);
    if (rc != ISAM_OK) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ISAM_ENODEV;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ISAM_ENODEV;

    isam_plan_s* p = new (std::nothrow) isam_plan_s();
    if (!p) return ISAM_ENOMEM;
    derive(p, g);
    p->device = dev;
    g_fail_alloc = 0;
    if (const char* env = std::getenv("ISAM_FAIL_ALLOC")) g_fail_alloc = std::atoi(env);
    if (const char* env = std::getenv("ISAM_LAT_C")) p->lat_c = std::atoi(env);
    if (const char* env = std::getenv("ISAM_LAT_CR")) p->lat_cr = std::atoi(env);
    // 1024 or 1280 lateral points and fewer than 2048 depth columns (over all slabs): 8-lane
    // tiles would leave CUs without a workgroup, so the complex passes take 4 lanes (update
    // pass at 1024 x 1024: 15.3 -> 13.1 us; at 1280 x 1024: 21.5 -> 17.0 us)
    if (p->lat_c == 0 && (p->nx == 1024 || p->nx == 1280) && (int64_t)p->ny * p->nk < 2048) p->lat_c = 4;
    const size_t full = (size_t)p->ncol * p->nk, half = (size_t)p->nhalf * p->nk;
    // forward NUFFT (ncol / 2 workgroups) plus the update pass (up to 2 nk per slab)
    p->red.maxBlocks = p->ncol + 2 * p->nk * p->ny + 2048;
    const int nsums = kPieces * 4 * kJ + (2 * kJ - 1);
    std::vector<isam::FwdPair> hp;
    build_columns(p, hp);
    p->npairs = (int)hp.size();
    rc = ISAM_OK;
    rc = rc ? rc : dalloc(&p->q2, p->ncol);
    rc = rc ? rc : dalloc(&p->Bl, p->ncol);
    rc = rc ? rc : dalloc(&p->pairs, hp.size());
    if (rc == ISAM_OK &&
        hipMemcpy(p->pairs, hp.data(), hp.size() * sizeof(isam::FwdPair), hipMemcpyHostToDevice) != hipSuccess)
        rc = ISAM_EHIP;
    if (p->ny > 1) {
        for (int L = 2; L <= 4; ++L) rc = rc ? rc : dalloc(&p->twY[L], fft_stage_len(p->ny, L));
        rc = rc ? rc : dalloc(&p->xs, full);
        rc = rc ? rc : dalloc(&p->xsh, half);
    }
    rc = rc ? rc : dalloc(&p->En, p->nk);
    rc = rc ? rc : dalloc(&p->sm, p->nk);
    rc = rc ? rc : dalloc(&p->wtab, kWtabEntries);
    rc = rc ? rc : dalloc(&p->twK, fft_stage_len(p->K, 4));
    rc = rc ? rc : dalloc(&p->twK8, fft_stage_len(p->K, 3));
    rc = rc ? rc : dalloc(&p->twN, fft_stage_len(p->nk, 4));
    rc = rc ? rc : dalloc(&p->Dn, p->nk);
    rc = rc ? rc : dalloc(&p->Pm, p->nk);
    for (int L = 2; L <= 4; ++L) rc = rc ? rc : dalloc(&p->twX[L], fft_stage_len(p->nx, L));
    rc = rc ? rc : dalloc(&p->wscratch, 2 * nsums);
    rc = rc ? rc : dalloc(&p->etahat, full);
    rc = rc ? rc : dalloc(&p->zh, half);
    rc = rc ? rc : dalloc(&p->rh, half);
    rc = rc ? rc : dalloc(&p->ghat, full);
    rc = rc ? rc : dalloc(&p->fista_hat, full);
    rc = rc ? rc : dalloc(&p->yhat, half);
    rc = rc ? rc : dalloc(&p->vec, full);
    rc = rc ? rc : dalloc(&p->sbuf, full);
    rc = rc ? rc : dalloc(&p->wbuf, full);
    rc = rc ? rc : dalloc(&p->zblk, full);
    rc = rc ? rc : dalloc(&p->red.partials, (size_t)p->red.maxBlocks * kRedSlots);
    rc = rc ? rc : dalloc(&p->red.sums, kRedSlots);
    // The two host records are mapped and coherent, so that a kernel can write them directly
    // (visible to the host once the stream has been synchronised).
    constexpr unsigned kHostFlags = hipHostMallocMapped | hipHostMallocCoherent;
    if (rc == ISAM_OK && hipHostMalloc((void**)&p->host_sums, kRedSlots * sizeof(double), kHostFlags) != hipSuccess)
        rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipMalloc((void**)&p->stop, sizeof(isam::StopState)) != hipSuccess) rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && hipHostMalloc((void**)&p->host_stop, sizeof(isam::StopState), kHostFlags) != hipSuccess)
        rc = ISAM_ENOMEM;
    if (rc == ISAM_OK && (hipHostGetDevicePointer((void**)&p->host_sums_dev, p->host_sums, 0) != hipSuccess ||
                          hipHostGetDevicePointer((void**)&p->host_stop_dev, p->host_stop, 0) != hipSuccess))
        rc = ISAM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    if (rc == ISAM_OK) rc = build_twiddles(p, s);
    if (rc == ISAM_OK) rc = build_calibrated_tables(p, s);
    if (rc == ISAM_OK) rc = check_stolt(p, s);
    if (rc != ISAM_OK) {
        release(p);
        return rc;
    }
    *out = p;
    return ISAM_OK;
}

extern "C" int isam_set_calibration(isam_plan_t p, double a2, double a3, double z_focus, void* stream) {
    if (!p) return ISAM_EINVAL;
    if (!std::isfinite(a2) || !std::isfinite(a3) || !std::isfinite(z_focus)) return ISAM_EINVAL;
    isam_geometry g = p->g;
    g.a2 = a2;
    g.a3 = a3;
    g.z_focus = z_focus;
    derive(p, &g);
    hipStream_t s = (hipStream_t)stream;
    int rc = build_calibrated_tables(p, s);
    if (rc == ISAM_OK && hipStreamSynchronize(s) != hipSuccess) rc = ISAM_EHIP;
    return rc;
}

extern "C" void isam_destroy(isam_plan_t p) {
    if (p) release(p);
}

extern "C" int isam_plan_dims(isam_plan_t p, int32_t* nx, int32_t* nk, int32_t* K) {
    if (!p) return ISAM_EINVAL;
    if (nx) *nx = p->nx;
    if (nk) *nk = p->nk;
    if (K) *K = p->K;
    return ISAM_OK;
}
