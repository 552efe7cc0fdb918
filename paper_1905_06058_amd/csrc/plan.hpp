// Internal plan state shared by the ISAM library's translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "isam.h"

namespace isam {

// Start/stop events the next pass kernel carries while isam_timing is on (set by the calling
// thread around each timed pass, null otherwise).  The runtime stamps them with the kernel's own
// begin and end, so a pass's time excludes the dispatch gaps around it.
struct PassEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local PassEvents g_pass_events;

}  // namespace isam

// Launch of a pass kernel: with the timing events of the pass when isam_timing has set them,
// else a plain launch.
#define ISAM_LAUNCH(KERNEL, GRID, BLOCK, LDS, S, ...)                                                  \
    do {                                                                                             \
        if (isam::g_pass_events.start)                                                               \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, S, isam::g_pass_events.start,            \
                                  isam::g_pass_events.stop, 0u, __VA_ARGS__);                        \
        else                                                                                         \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, S, __VA_ARGS__);                            \
    } while (0)

namespace isam {

constexpr int kJ = 6;             // interpolation taps (the only J built)
constexpr int kPieces = 32;       // piecewise-cubic pieces of the min-max weight table over tau in [0,1)
// float2 coefficients c0..c3 per tap; a piece's 6 taps are followed by 2 pad entries (26 float2 =
// 52 dwords per piece, so lanes reading different pieces hit different LDS banks)
constexpr int kWtabPiece = kJ * 4 + 2;
constexpr int kWtabEntries = kPieces * kWtabPiece;
constexpr int kRedSlots = 8;      // scalars per workgroup in reduction partials

// Columns of one forward-NUFFT workgroup.  mode 0: a and b are Hermitian partners
// (a stored at half row ha; hb >= 0 if b is stored too); mode 1: a and b are two
// self-paired columns (rows ha, hb); mode 2: a alone, self-paired.
struct FwdPair {
    int a, b, ha, hb, mode;
};

// Constant arguments of the per-column NUFFT kernels.
struct NufftArgs {
    int nx, nk, K;
    int mi;                 // integer part of the focal row (circular shift of the depth buffer)
    int has_frac;           // nonzero if the focal row has a fractional part
    double mr_over_K;       // fractional focal row / K (per-point phase exp(-2 pi i m_r t / K))
    double kc, dk;          // k_n = kc + (n - nk/2) dk
    double cT;              // Stolt grid position t = kz * cT, cT = dz K / (2 pi)
    // q = 0 (kz = 2k): t_n = t0 + osf (n - nk/2) exactly, split once into floor(t0) and t0 - floor(t0)
    int f0;
    float tau0;
    double t0;
    const double* q2;       // [nx] q_l^2 (FP64)
    const float* Bl;        // [nx] beam filter exp(-q^2 w0^2 / 8)
    const float2* En;       // [nk] e^{i phi(k_n)} e^{2 i k_n z_f} / sqrt(nz)
    const float* sm;        // [nk] Kaiser-Bessel scaling at depth index i = m + nz/2
    const float2* wtab;     // [kPieces][kJ][4] cubic coefficients of the weights (focus-phased)
    const float2* tw;       // staged twiddles of the K-point FFT, radices up to 16
    const float2* tw8;      // staged twiddles of the K-point FFT, radices up to 8
    const int* stop;        // solver stop flag (non-zero: return at once), or null
    int ncol;               // lateral-frequency columns (nx for a B-scan, nx * ny for a volume)
    int nhalf;              // columns of the Hermitian half arrays (nx/2 + 1, times ny)
    const FwdPair* pairs;   // NUFFT (forward and adjoint): column pair of each workgroup
    // adjoint only: with step_eta set, the output is the FISTA gradient step
    // step_eta - gstep * g_hat instead of g_hat
    const float2* step_eta = nullptr;
    float gstep = 0.f;
};


// Device-side state of the relative-residual stop rule (Eq. 15): iteration at which it
// held (0: not yet), status (ISAM_ENONFINITE on non-finite norms), last r_r.
struct StopState {
    int iter;
    int status;
    double rel_res;
};

// Step record of the FISTA update pass (Alg. 1, Eq. 14): step 1/L, lambda, momentum
// weight beta, whether to form the Eq. 15 norms.
struct FistaStep {
    float step, lam, beta;
    int norms;
    const int* stop;     // solver stop flag (non-zero: return at once), or null
    int pre = 0;         // ghat already holds eta_hat - step * g_hat (formed by the adjoint)
};

// Operands of one scan in a batched NUFFT pass (forward: in = eta_hat, in2 = F(y) or null,
// out = Z or the residual spectrum, partials = ||r||^2 partials or null; adjoint: in =
// residual half spectrum, out = g_hat).  nblk: the scan's workgroups in the pass.
struct NuScan {
    NufftArgs a;
    const float2* in;
    const float2* in2;
    float2* out;
    float* partials;
    int nblk;
};

// Operands of one scan in a batched lateral pass.  c2c / c2r / r2c: in -> out.  FISTA
// update: out = eta_hat (read and written), in = g_hat, z, w (or null), partials, and the
// scan's step record fs (its beta is replaced by the batch's).  tw: the scan's lateral
// twiddle table for the pass's radix cap; ntiles: the scan's workgroups in the pass.
struct LatScan {
    const void* in;
    void* out;
    float2* z;
    const float* w;
    float* partials;
    const float2* tw;
    FistaStep fs;
    int nk;
    int ntiles;
};

struct Reduce {
    float* partials;        // [maxBlocks][kRedSlots]
    double* sums;           // [kRedSlots] final FP64 values (device)
    int maxBlocks;
};

}  // namespace isam

struct isam_plan_s {
    isam_geometry g;
    int device;
    int nx, nk, K, nh;
    int ny = 1;                   // A-scan rows of a volume (1 for a B-scan)
    int ncol = 0, nhalf = 0;      // lateral-frequency columns: nx * ny, (nx/2 + 1) * ny
    int npairs = 0;               // NUFFT workgroups
    double kc, band, dk, dz, cT, beta, mf;
    int mi;
    double mr;
    double t0;                    // Stolt position 2 kc cT of the centre sample at q = 0
    int f0;                       // floor(t0)
    int lat_c = 0;                // lateral tile width of complex passes (lanes); 0 = default
    int lat_cr = 0;               // lateral tile width of real passes (lanes); 0 = default
    int lat_cy = 0;               // tile width of the y transform of a volume (lanes); 0 = default

    // tables (device)
    double* q2 = nullptr;
    float* Bl = nullptr;
    float2* En = nullptr;
    float* sm = nullptr;
    float2* wtab = nullptr;
    float2* twK = nullptr;
    float2* twK8 = nullptr;
    float2* twX[5] = {};          // staged lateral twiddles for radix caps 2^2, 2^3, 2^4 (index = log2 cap)
    float2* twN = nullptr;        // staged twiddles of the nk-point FFT (direct image), radices up to 16
    float2* Dn = nullptr;         // [nk] e^{-i phi(k_n)} (dispersion compensation of the direct image)
    float2* Pm = nullptr;         // [nk] per-row phase of the direct image, divided by sqrt(nk)
    float2* twY[5] = {};          // the same for the y transform of a volume
    isam::FwdPair* pairs = nullptr;   // [npairs] NUFFT column pairs
    double* wscratch = nullptr;   // FP64 scratch of the weight-table build

    // workspace (device)
    // lateral-frequency arrays, column-blocked (see blk in common.hpp)
    float2* etahat = nullptr;     // [nx][nk] lateral spectrum of the operator input
    float2* zh = nullptr;         // [nh][nk] Hermitian half of the forward spectrum
    float2* rh = nullptr;         // [nh][nk] half spectrum of a real residual
    float2* ghat = nullptr;       // [nx][nk] lateral spectrum of the adjoint output
    float2* fista_hat = nullptr;  // [nx][nk] FISTA momentum point in lateral frequency
    float2* yhat = nullptr;       // [nh][nk] lateral spectrum of the measured spectra (FISTA)
    float2* vec = nullptr;        // [nx][nk] power-iteration vector
    float* sbuf = nullptr;        // [nx][nk] real spectra scratch (FISTA: blocked data y)
    float* wbuf = nullptr;        // [nx][nk] blocked l1 weights of FISTA
    float2* zblk = nullptr;       // [nx][nk] blocked FISTA iterate z
    float2* xs = nullptr;         // volume only: [ny] slabs of [nx][nk] x-spectra (blocked per slab)
    float2* xsh = nullptr;        // volume only: [ny] slabs of [nh][nk] half x-spectra (blocked per slab)
    isam::Reduce red;
    double* host_sums = nullptr;  // pinned host copy of red.sums
    isam::StopState* stop = nullptr;       // device stop-rule state of the solver
    isam::StopState* host_stop = nullptr;  // pinned host copy
    // device addresses of the two pinned host records, which the solver's last kernel writes
    double* host_sums_dev = nullptr;
    isam::StopState* host_stop_dev = nullptr;
    double* hist = nullptr;       // per-iteration FISTA history [cap][3] (device), grown on demand
    int hist_cap = 0;

    // per-pass timing (isam_timing)
    int timing_on = 0;
    int tev_used = 0;
    int tev_cap = 0;
    hipEvent_t* tev = nullptr;    // event pairs
    int* ttag = nullptr;          // pass of each pair
    hipStream_t tstream = nullptr;
    double tms[ISAM_NPASS] = {};
    int64_t tcnt[ISAM_NPASS] = {};

    isam::NufftArgs nufft_args() const;
};

namespace isam {

// launchers (return hipError_t of the launch)
hipError_t lat_c2c(const isam_plan_s* p, const float2* in, float2* out, int sign, hipStream_t s);
// y transform of a volume (length ny) over ncols columns: sign -1 row-major -> blocked, +1 back.
hipError_t lat_c2c_y(const isam_plan_s* p, const float2* in, float2* out, int ncols, int sign, hipStream_t s);
hipError_t lat_c2r(const isam_plan_s* p, const float2* zh, float* s_out, hipStream_t st);
hipError_t lat_r2c(const isam_plan_s* p, const float* r, float2* rh, hipStream_t st);
// FISTA update pass; see solver.hip
hipError_t lat_fista(const isam_plan_s* p, float2* eta_hat, const float2* ghat, float2* z,
                     const float* w, FistaStep fs, float* partials, hipStream_t st);
int lat_blocks(const isam_plan_s* p, int kind);   // number of workgroups of a lateral pass
int lat_l(const isam_plan_s* p);                  // radix cap (log2) of the lateral FFT

// Raise a kernel's dynamic LDS limit to bytes (needed above 64 KiB), once per kernel and device.
void set_max_lds(const void* kern, size_t bytes);

// Forward Stolt NUFFT: zh = Z (yhat null) or the residual spectrum Z - yhat; ||.||^2 partials
// (Parseval weights) per workgroup into partials slot 0 if partials is non-null.
hipError_t nufft_fwd(const isam_plan_s* p, const float2* etahat, const float2* yhat, float2* zh, float* partials,
                     hipStream_t s, const int* stop = nullptr);
// Batched passes over one group of scans (same lateral length nx, or same depth FFT length
// K).  recs: device records indexed by batch scan; map: device block map (scan, workgroup of
// the scan) with nblk entries; sel: requested lateral tile width (lanes).
hipError_t lat_c2c_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, int sign, hipStream_t s);
hipError_t lat_c2r_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, hipStream_t s);
hipError_t lat_r2c_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, hipStream_t s);
hipError_t lat_fista_batch(int nx, int sel, int norms, const LatScan* recs, const int2* map, int nblk,
                           const float* beta, hipStream_t s);
hipError_t nufft_fwd_batch(int K, const NuScan* recs, const int2* map, int nblk, hipStream_t s);
hipError_t nufft_adj_batch(int K, const NuScan* recs, const int2* map, int nblk, hipStream_t s);
int lat_tile(int nx, int sel, int real);        // lanes per tile built for (nx, sel)
int lat_radix_cap(int nx, int sel, int real);   // radix cap (log2) of that configuration
// FISTA set-up and output steps shared by the single and batched solvers (solver.hip).
// zero_state: zero both state arrays, for a start from eta^1 = z^0 = 0 (false: the caller
// restores a saved state, or has its first iteration clear them, see fista_first).  Also
// resets the plan's device stop state.
int fista_prepare(isam_plan_t p, const float* y, const float* w, hipStream_t s, bool zero_state = true);
// convert: write z^k into out (false: the caller has done so).
int fista_finish(isam_plan_t p, double L, int add_residual, float2* out, hipStream_t s, bool convert = true);
// Whether a lateral length has built kernels (powers of two up to 2048 and 3, 5, 7 times
// powers of two from 192 up to 1792).
bool lat_supported(int nx);
int nufft_fwd_blocks(const isam_plan_s* p);
int nufft_adj_blocks(const isam_plan_s* p);
// Adjoint Stolt NUFFT: ghat = g_hat, or with step_eta the gradient step step_eta - gstep g_hat.
hipError_t nufft_adj(const isam_plan_s* p, const float2* rh, float2* ghat, hipStream_t s,
                     const int* stop = nullptr, const float2* step_eta = nullptr, float gstep = 0.f);
hipError_t nufft_calgrad(const isam_plan_s* p, const float2* etahat, const float2* ghalf, float* partials,
                         hipStream_t s);
// Device check, with the kernels' own Stolt arithmetic, of the two bounds the adjoint's
// single-writer slots rely on; writes one flag per (column, chunk) into partials.
hipError_t nufft_check(const isam_plan_s* p, float* partials, int* nslots, hipStream_t s);
// Plan inspection (isam_plan_stolt, isam_plan_weights).
hipError_t inspect_stolt(const isam_plan_s* p, int col, int* fl, float* tau, hipStream_t s);
hipError_t inspect_weights(const isam_plan_s* p, const float* tau, int n, float2* out, hipStream_t s);
// Direct image of Eq. 9 (per A-scan dispersion compensation and inverse transform).
hipError_t direct_image(const isam_plan_s* p, const float* y, float2* out, hipStream_t s);

}  // namespace isam
